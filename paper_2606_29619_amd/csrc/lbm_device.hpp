// lbm_device.hpp -- gfx950 device code of the porous-media lattice Boltzmann step.
//
// The method is the one-domain scheme of Gusev & Karlin (arXiv 2606.29619): product-form
// porosity-scaled equilibrium (Sec. 3.2, eqs. 1d_scaled_eq, prod_form), Relax-to-Force shifted
// equilibrium with the extended-equilibrium and bulk-viscosity corrections (eqs. xi_alpha_*,
// P_aa_*, ex_corr, eta_corr), collide-and-stream with per-cell relaxation (Sec. 3.3, eqs.
// dicrete_scheme, momentum_rate, beta_def), the closed-form drag solve and the
// variable-porosity viscous correction (eqs. v_(0), v_(1), v_final, accel,
// porosity_correction_expanded).
//
// Storage: structure-of-arrays populations f[i][n], n = x + nx*(y + ny*z), one in-place buffer
// streamed with the AA pattern:
//   phase 0 (natural layout): cell n reads f_i from slot (i, n) and writes its post-collision
//            value to slot (opp(i), n);
//   phase 1 (swapped layout): cell n reads f_i from slot (opp(i), n - c_i) and writes to slot
//            (i, n + c_i).
// Halfway bounce-back only touches phase 1: a population whose source (n - c_i) is solid is the
// cell's own reflected value in slot (i, n), and one whose destination (n + c_i) is solid is
// written back to slot (opp(i), n).  Every thread reads and writes the same set of slots, so
// the update is race-free in place.  Every axis wraps periodically.
//
// Addressing: every array plane (one population, one scalar field, or the packed four-value
// moment records) holds fewer than 2^32 bytes, so a thread addresses it with a 32-bit byte offset added to a uniform 64-bit base (the scalar-base + vector-offset form of
// the global memory instructions).  The periodic neighbours of a cell are precomputed once
// per thread (three x positions, nine y/z row bases).
//
// Floating point: built with -ffp-contract=off.  In FP64 every expression is evaluated exactly
// as written, in the order of the CPU reference, so FP64 results agree bit for bit.  In FP32 a
// quotient a/b is a * rcp(b) and a square root is the hardware one (both within 1 ulp): the FP32
// path is checked against the FP64 reference with a stated tolerance, not bitwise.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace lbm {

template <int D>
struct Lat;

// D2Q9 in the numbering of the paper's wall example (Sec. 3.4.1).
template <>
struct Lat<2> {
    static constexpr int Q = 9;
    static constexpr int c[9][3] = {{0, 0, 0},  {1, 0, 0},   {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, 1, 0},  {-1, -1, 0}, {1, -1, 0}};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
};

// D3Q27: rest, faces, edges, corners; opposite pairs adjacent.
template <>
struct Lat<3> {
    static constexpr int Q = 27;
    static constexpr int c[27][3] = {
        {0, 0, 0},   {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
        {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},
        {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1},  {0, -1, 1},  {1, 1, 1},  {-1, -1, -1},
        {1, 1, -1},  {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};
    static constexpr int opp[27] = {0,  2,  1,  4,  3,  6,  5,  8,  7,  10, 9,  12, 11, 14,
                                    13, 16, 15, 18, 17, 20, 19, 22, 21, 24, 23, 26, 25};
};

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void unroll(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        unroll<B + 1, E>(f);
    }
}

struct Grid {
    int nx, ny, nz;
    uint32_t N;  // cells; 4 N sizeof(T) < 2^32
};

template <typename T>
struct Phys {
    T RT;          // lattice temperature
    T omr;         // 1 - 3 RT
    T nu_ref;      // nu_eff(eps) = nu_ref * eps^nu_pow
    T eta;         // effective bulk viscosity (Phi^eta)
    T two_over_D;  // 2 / D
    T b[3];        // body acceleration
    T rho0;        // reference density of the 16-bit population shift
    int nu_pow;    // -1, 0, 1
    int eta_on;    // Phi^eta switched on
    int shift_porous;  // 16-bit shift base rho0 eps(src) (1) or rho0 (0)
    const T *deps;     // analytic porosity derivatives: planes of dN values, grad eps (D planes)
                       // then the Hessian's upper triangle row by row; null: central differences
    uint32_t dN;       // plane stride of deps (cells)
};

// Plane of the Hessian entry (a, b), a <= b, among the analytic derivative planes.
template <int D>
constexpr int hess_plane(int a, int b) {
    return D + a * D - a * (a - 1) / 2 + (b - a);
}

// ---- arithmetic policy -------------------------------------------------------------------
__device__ __forceinline__ double dv(double a, double b) { return a / b; }
__device__ __forceinline__ float dv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// Correctly rounded quotient, for rho = S / eps: eps rho then scales the equilibria, whose sum
// is the cell's mass after collision, and rcp's rounding is not symmetric (FP32 runs lost
// mass steadily with it).
__device__ __forceinline__ double div_rn(double a, double b) { return a / b; }
__device__ __forceinline__ float div_rn(float a, float b) { return a / b; }
__device__ __forceinline__ double sq(double x) { return sqrt(x); }
__device__ __forceinline__ float sq(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---- memory access -------------------------------------------------------------------------
// Element `idx` of a plane starting at `base`: 32-bit byte offset on a uniform base.
template <typename T>
__device__ __forceinline__ const T *at(const T *base, uint32_t idx) {
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                       idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T *at(T *base, uint32_t idx) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T ld(const T *base, uint32_t idx) {
    return *at(base, idx);
}

// Populations stream through once per kernel.  In the natural-layout phase each thread touches
// only its own cell, and the accesses are non-temporal (the caches are left to the reused
// moment and porosity fields).  In the swapped phase the x-shifted accesses (c_x != 0) of
// neighbouring lanes and waves share cache lines, so they go through the caches normally, while
// those with c_x = 0 cover whole lines of one wave and stay non-temporal (256^3 box: FP32 step
// 1.236 -> 1.218 ms, FP32 lagged pass 1.050 -> 1.026 ms; the moment pass with every load of the
// swapped phase non-temporal was 0.6 % slower than with this rule).
template <bool NT, typename T>
__device__ __forceinline__ T ld_pop(const T *base, uint32_t idx) {
    if constexpr (NT) return __builtin_nontemporal_load(at(base, idx));
    else return *at(base, idx);
}
template <bool NT, typename T>
__device__ __forceinline__ void st_pop(T *base, uint32_t idx, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, at(base, idx));
    else *at(base, idx) = v;
}

template <typename T>
__device__ __forceinline__ const T *plane(const T *f, int i, uint32_t N) {
    return f + (size_t)i * N;
}
template <typename T>
__device__ __forceinline__ T *plane(T *f, int i, uint32_t N) {
    return f + (size_t)i * N;
}

__device__ __forceinline__ int wrap1(int x, int k, int n) {
    // x + k on a periodic axis of length n, for k in {-1, 0, 1}
    if (k > 0) return x + 1 == n ? 0 : x + 1;
    if (k < 0) return x == 0 ? n - 1 : x - 1;
    return x;
}

__device__ __forceinline__ int wrapk(int x, int k, int n) {
    int r = (x + k) % n;
    return r < 0 ? r + n : r;
}

// Periodic neighbourhood of one cell: cell index of (x + cx, y + cy, z + cz), |c| <= 1.
template <int D>
struct Nbr {
    uint32_t xs[3];
    uint32_t row[3][3];
    int x, y, z;
    // The row bases use one multiply per axis: the +-1 neighbours differ from the centre by the
    // row (plane) stride, or by the wrapped distance on the periodic seam.
    __device__ __forceinline__ void init(const Grid &g, int x_, int y_, int z_) {
        x = x_;
        y = y_;
        z = z_;
        const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
        xs[0] = (uint32_t)(x == 0 ? g.nx - 1 : x - 1);
        xs[1] = (uint32_t)x;
        xs[2] = (uint32_t)(x + 1 == g.nx ? 0 : x + 1);
        const uint32_t sy = nx * (ny - 1u);
        const uint32_t r1 = nx * (uint32_t)y;
        const uint32_t ry[3] = {y == 0 ? r1 + sy : r1 - nx, r1, y + 1 == g.ny ? r1 - sy : r1 + nx};
        uint32_t rz[3] = {0u, 0u, 0u};
        if constexpr (D == 3) {
            const uint32_t pl = nx * ny;
            const uint32_t sz = pl * ((uint32_t)g.nz - 1u);
            const uint32_t z1 = pl * (uint32_t)z;
            rz[0] = z == 0 ? z1 + sz : z1 - pl;
            rz[1] = z1;
            rz[2] = z + 1 == g.nz ? z1 - sz : z1 + pl;
        } else {
            rz[1] = nx * ny * (uint32_t)z;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (D == 2 && k != 1) continue;
                row[j][k] = ry[j] + rz[k];
            }
    }
    __device__ __forceinline__ uint32_t at(int cx, int cy, int cz) const {
        return xs[cx + 1] + row[cy + 1][cz + 1];
    }
    __device__ __forceinline__ uint32_t self() const { return at(0, 0, 0); }
    // A copy whose row and column indices the compiler cannot prove equal to these.  In the
    // swapped phase the population slots are the stencil neighbours whose porosity and records
    // were read first; addresses built from the copy are recomputed (one add each) next to the
    // population loads and stores instead of being held in registers from those stencil loads
    // (FP32 lagged pass 170 -> 121 registers, 16-bit collision 124 -> 112).  The empty asm
    // statements emit no instruction.
    __device__ __forceinline__ Nbr opaque() const {
        Nbr r = *this;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            asm volatile("" : "+v"(r.xs[j]));
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (D == 2 && k != 1) continue;
                asm volatile("" : "+v"(r.row[j][k]));
            }
        }
        return r;
    }
    // Neighbour along axis a at offset k (|k| <= 2).
    __device__ __forceinline__ uint32_t axis(const Grid &g, int a, int k) const {
        if (k == 1 || k == -1) {
            return a == 0 ? at(k, 0, 0) : (a == 1 ? at(0, k, 0) : at(0, 0, k));
        }
        int c[3] = {x, y, z};
        const int n = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
        c[a] = wrapk(c[a], k, n);
        return (uint32_t)c[0] + (uint32_t)g.nx * ((uint32_t)c[1] + (uint32_t)g.ny * (uint32_t)c[2]);
    }
};

// ------------------------------------------------------------------------------------------
// Porosity of the cell's periodic 3x3(x3) neighbourhood.  The tiled kernels stage the porosity
// of their tile and its one-cell halo in LDS once (coalesced rows) and read every neighbour
// from there; the other kernels read global memory.  at(dx, dy, dz) with |d| <= 1.
// ------------------------------------------------------------------------------------------
template <int D, typename T>
struct EpsGlobal {
    const T *eps;
    const Nbr<D> *nb;
    __device__ __forceinline__ T at(int dx, int dy, int dz) const {
        return ld(eps, nb->at(dx, dy, dz));
    }
};

template <int D, typename T>
struct EpsTile {
    // the largest halo: a 256 x 1 tile, (256 + 2) x 3 rows per plane, 3 planes in 3D
    static constexpr int kSize = D == 3 ? 258 * 3 * 3 : 258 * 3;
    const T *lds;    // the cell's own entry
    int row, plane;  // strides: halo row length (tx + 2) and plane size (tx + 2)(ty + 2)
    __device__ __forceinline__ T at(int dx, int dy, int dz) const {
        return lds[(D == 3 ? dz * plane : 0) + dy * row + dx];
    }
};

// Stage the porosity of the tile with origin (x0, y0) in plane z0 and its periodic halo.
// Every thread of the workgroup takes part; the caller synchronises afterwards.
template <int D, typename T>
__device__ __forceinline__ void stage_eps(const T *__restrict__ eps, const Grid &g, int tx,
                                          int ty, int x0, int y0, int z0, T *lds) {
    const int row = tx + 2, rows = ty + 2;
    constexpr int planes = D == 3 ? 3 : 1;
    const int total = planes * rows * row;
    const int nx = g.nx, ny = g.ny;
    // periodic coordinate c >= -1: at most one correction except on grids narrower than the
    // tile
    auto wrap = [](int c, int n) {
        if (c < 0) c += n;
        while (c >= n) c -= n;
        return c;
    };
    // Element e of the halo (row-major: plane, row, column) goes to lds[e].  Every load of the
    // thread is issued before the first LDS write, so they are in flight together (a loop over
    // halo rows waited for each load in turn: 256^3 box, FP16 moment pass 0.439 -> 0.305 ms,
    // FP16 lagged pass 1.144 -> 0.882 ms).
    constexpr int kIt = (EpsTile<D, T>::kSize + 255) / 256;
    const float inv_row = 1.0f / (float)row;
    T v[kIt];
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
        const int e = (int)threadIdx.x + 256 * k;
        v[k] = T(0);
        if (e < total) {
            int p = (int)((float)e * inv_row);  // row of the halo, corrected to floor(e / row)
            if (p * row > e) --p;
            else if ((p + 1) * row <= e) ++p;
            const int px = e - p * row;
            const int pz = D == 3 ? (p >= 2 * rows ? 2 : (p >= rows ? 1 : 0)) : 0;
            const int py = p - pz * rows;
            const int zz = D == 3 ? wrap(z0 + pz - 1, g.nz) : z0;
            const int yy = wrap(y0 + py - 1, ny);
            const uint32_t base = (uint32_t)nx * ((uint32_t)yy + (uint32_t)ny * (uint32_t)zz);
            v[k] = ld(eps, base + (uint32_t)wrap(x0 + px - 1, nx));
        }
    }
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
        const int e = (int)threadIdx.x + 256 * k;
        if (e < total) lds[e] = v[k];
    }
}

// ------------------------------------------------------------------------------------------
// Population storage formats.  FP64 and FP32 slots hold f-bar itself.  The 16-bit formats
// (FP16, BF16) hold the deviation from a shift, scaled per direction,
//     slot = (f-bar_i - sigma_i) * 2^k_i,    sigma_i = base * w_i,
// with base = rho0 (shift by the lattice weights) or base = rho0 eps(src) (porous shift), where
// src is the cell whose collision produced the value: a resting porous cell holds eps rho0 w_i,
// so the porous shift leaves only the flow's own deviation to the 16-bit value.  2^k_i is the
// largest power of two not above 2^12 / w_i: deviations down to ~1e-5 of a weight stay in the
// FP16 normal range, and the scaling is exact, so a value decoded in FP64 re-encodes to the
// same bits.  Arithmetic stays FP32.
// ------------------------------------------------------------------------------------------
template <typename P>
struct PopFmt {
    static constexpr bool shifted = false;
};
template <>
struct PopFmt<_Float16> {
    static constexpr bool shifted = true;
    __device__ static __forceinline__ float dec(_Float16 h) { return (float)h; }
    __device__ static __forceinline__ _Float16 enc(float x) { return (_Float16)x; }
};
template <>
struct PopFmt<__bf16> {
    static constexpr bool shifted = true;
    __device__ static __forceinline__ float dec(__bf16 h) { return (float)h; }
    __device__ static __forceinline__ __bf16 enc(float x) { return (__bf16)x; }
};

// Lattice weight of direction I: the product over axes of 2/3 (c = 0) or 1/6 (c = +-1), i.e.
// the rest-state factors of the product-form equilibrium.
template <int D, int I>
__device__ __forceinline__ constexpr float weight() {
    using L = Lat<D>;
    float w = 1.0f;
    for (int a = 0; a < D; ++a) w *= L::c[I][a] == 0 ? (2.0f / 3.0f) : (1.0f / 6.0f);
    return w;
}
// 2^k_I <= 2^12 / w_I (1 / w_I is a product of 3/2 and 6, computed exactly).
template <int D, int I>
__device__ __forceinline__ constexpr float enc_scale() {
    using L = Lat<D>;
    float r = 4096.0f;
    for (int a = 0; a < D; ++a) r *= L::c[I][a] == 0 ? 1.5f : 6.0f;
    float p = 1.0f;
    while (p * 2.0f <= r) p *= 2.0f;
    return p;
}

// Shift sigma_I = base * w_I of a value produced by a cell of porosity e_src (16-bit formats;
// FP32 product).
template <int D, int I, typename P, typename T>
__device__ __forceinline__ float shift_sigma(T e_src, const Phys<T> &ph) {
    if constexpr (!PopFmt<P>::shifted) {
        return 0.0f;
    } else {
        const float base = ph.shift_porous ? ph.rho0 * e_src : ph.rho0;
        return base * weight<D, I>();
    }
}

// Value of a slot in arithmetic type A (FP32 in the kernels; FP64 for exact checkpoints).
template <int D, int I, typename A, typename P>
__device__ __forceinline__ A decode(P raw, float sigma) {
    if constexpr (!PopFmt<P>::shifted) {
        return (A)raw;
    } else {
        constexpr float dscale = 1.0f / enc_scale<D, I>();
        return (A)sigma + (A)PopFmt<P>::dec(raw) * (A)dscale;
    }
}
template <int D, int I, typename P, typename A>
__device__ __forceinline__ P encode(A v, float sigma) {
    if constexpr (!PopFmt<P>::shifted) {
        return (P)v;
    } else {
        constexpr float escale = enc_scale<D, I>();
        return PopFmt<P>::enc((float)((v - (A)sigma) * (A)escale));
    }
}

// ------------------------------------------------------------------------------------------
// AA-pattern population access
// ------------------------------------------------------------------------------------------
// Cell whose collision produced the population f_I found at cell n: the upstream cell
// n - c_I, or n itself when that cell is solid (the value was bounced back at n).  This holds
// for the natural layout (read in phase 0) and for the swapped one (read in phase 1).
template <int D, bool SOLIDS, int I>
__device__ __forceinline__ uint32_t source_cell(const uint8_t *__restrict__ mask,
                                                const Nbr<D> &nb) {
    using L = Lat<D>;
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    if constexpr (cx == 0 && cy == 0 && cz == 0) {
        return nb.self();
    } else {
        const uint32_t s = nb.at(-cx, -cy, -cz);
        if constexpr (SOLIDS) {
            if (mask[s]) return nb.self();
        }
        return s;
    }
}

// Raw slot holding f_I of cell n (AA pattern, halfway bounce-back in phase 1).
template <int D, bool SOLIDS, int PH, int I, typename P>
__device__ __forceinline__ P load_raw(const P *__restrict__ f, const uint8_t *__restrict__ mask,
                                      const Grid &g, const Nbr<D> &nb) {
    using L = Lat<D>;
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    const uint32_t n = nb.self();
    constexpr bool NT = PH == 0 || cx == 0;
    if constexpr (PH == 0 || (cx == 0 && cy == 0 && cz == 0)) {
        return ld_pop<NT>(plane(f, I, g.N), n);
    } else {
        const uint32_t s = nb.at(-cx, -cy, -cz);
        if constexpr (SOLIDS) {
            if (mask[s]) return ld_pop<NT>(plane(f, I, g.N), n);
        }
        return ld_pop<NT>(plane(f, L::opp[I], g.N), s);
    }
}

// Shift of the f_I found at cell n (0 for FP64/FP32 storage): the porosity of its source cell,
// the upstream neighbour n - c_I or n itself after a bounce-back.
template <int D, bool SOLIDS, int I, typename P, typename T, typename E>
__device__ __forceinline__ float load_sigma(const uint8_t *__restrict__ mask, const E &ev,
                                            const Phys<T> &ph, const Nbr<D> &nb) {
    if constexpr (!PopFmt<P>::shifted) {
        return 0.0f;
    } else {
        using L = Lat<D>;
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        if (!ph.shift_porous) return shift_sigma<D, I, P>(T(1), ph);
        const bool own = (cx == 0 && cy == 0 && cz == 0) ||
                         (SOLIDS && source_cell<D, SOLIDS, I>(mask, nb) == nb.self());
        return shift_sigma<D, I, P>(own ? ev.at(0, 0, 0) : ev.at(-cx, -cy, -cz), ph);
    }
}

template <int D, bool SOLIDS, int PH, int I, typename T, typename P, typename E>
__device__ __forceinline__ T load_pop(const P *__restrict__ f, const uint8_t *__restrict__ mask,
                                      const E &ev, const Phys<T> &ph, const Grid &g,
                                      const Nbr<D> &nb) {
    const P raw = load_raw<D, SOLIDS, PH, I>(f, mask, g, nb);
    return decode<D, I, T>(raw, load_sigma<D, SOLIDS, I, P>(mask, ev, ph, nb));
}

// Store of the post-collision f_I of the cell; base is the cell's own shift base
// (rho0 or rho0 eps(n)) for the 16-bit formats.
template <int D, bool SOLIDS, int PH, int I, typename T, typename P>
__device__ __forceinline__ void store_pop(P *__restrict__ f, const uint8_t *__restrict__ mask,
                                          const Grid &g, const Nbr<D> &nb, T val, float base) {
    using L = Lat<D>;
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    const uint32_t n = nb.self();
    constexpr bool NT = PH == 0 || cx == 0;
    const P raw = encode<D, I, P>(val, base * weight<D, I>());
    if constexpr (PH == 0 || (cx == 0 && cy == 0 && cz == 0)) {
        st_pop<NT>(plane(f, L::opp[I], g.N), n, raw);
    } else {
        const uint32_t d = nb.at(cx, cy, cz);
        if constexpr (SOLIDS) {
            if (mask[d]) {
                st_pop<NT>(plane(f, L::opp[I], g.N), n, raw);
                return;
            }
        }
        st_pop<NT>(plane(f, I, g.N), d, raw);
    }
}

// Shift base of the cell itself (porosity e0) for store_pop.
template <typename P, typename T>
__device__ __forceinline__ float own_base(T e0, const Phys<T> &ph) {
    if constexpr (!PopFmt<P>::shifted) return 0.0f;
    else return ph.shift_porous ? ph.rho0 * e0 : ph.rho0;
}

// ------------------------------------------------------------------------------------------
// Per-cell coefficients
// ------------------------------------------------------------------------------------------
template <typename T>
struct Visc {
    T nu, dnu, beta;
};

// nu_eff(eps) = nu_ref eps^p and its derivative; beta from eq. (nu_eff_def) with dt = 1.
template <typename T>
__device__ __forceinline__ Visc<T> viscosity(const Phys<T> &ph, T e) {
    Visc<T> r;
    if (ph.nu_pow == -1) {
        r.nu = dv(ph.nu_ref, e);
        r.dnu = dv(-ph.nu_ref, e * e);
    } else if (ph.nu_pow == 1) {
        r.nu = ph.nu_ref * e;
        r.dnu = ph.nu_ref;
    } else {
        r.nu = ph.nu_ref;
        r.dnu = T(0);
    }
    r.beta = dv(T(1), T(1) + dv(T(2) * r.nu, ph.RT));
    return r;
}

// Component A of grad eps at cell n: the analytic input (AD) or the central difference.
// The choice is a template parameter: a run-time branch here costs the differenced kernels
// their register allocation (arrays of the stencil work spill to scratch).
template <int A, bool AD, typename T, typename E>
__device__ __forceinline__ T eps_gradient(const E &ev, const Phys<T> &ph, uint32_t n) {
    if constexpr (AD) {
        return ld(plane(ph.deps, A, ph.dN), n);
    } else {
        constexpr int px = A == 0, py = A == 1, pz = A == 2;
        return (ev.at(px, py, pz) - ev.at(-px, -py, -pz)) * T(0.5);
    }
}

// Porosity gradient and Hessian of cell n: the analytic inputs (AD), else central differences
// (eps is defined on every cell), the mixed derivatives from the four diagonal neighbours,
// computed once for a < b.
template <int D, bool AD, typename T, typename E>
__device__ __forceinline__ void porosity_derivatives(const E &ev, const Phys<T> &ph, uint32_t n,
                                                     T e0, T ge[3], T H[3][3]) {
    if constexpr (AD) {
        unroll<0, D>([&](auto ia) {
            constexpr int a = decltype(ia)::value;
            ge[a] = ld(plane(ph.deps, a, ph.dN), n);
            unroll<a, D>([&](auto ib) {
                constexpr int b = decltype(ib)::value;
                const T h = ld(plane(ph.deps, hess_plane<D>(a, b), ph.dN), n);
                H[a][b] = h;
                H[b][a] = h;
            });
        });
        return;
    }
    unroll<0, D>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        constexpr int px = a == 0, py = a == 1, pz = a == 2;
        const T ep = ev.at(px, py, pz);
        const T em = ev.at(-px, -py, -pz);
        ge[a] = (ep - em) * T(0.5);
        H[a][a] = (ep - T(2) * e0) + em;
    });
    unroll<0, D>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        unroll<a + 1, D>([&](auto ib) {
            constexpr int b = decltype(ib)::value;
            // offsets of the diagonal neighbour (ka along a, kb along b)
            constexpr int ax0 = a == 0, ay0 = a == 1, az0 = a == 2;
            constexpr int bx0 = b == 0, by0 = b == 1, bz0 = b == 2;
            const T pp = ev.at(ax0 + bx0, ay0 + by0, az0 + bz0);
            const T pm = ev.at(ax0 - bx0, ay0 - by0, az0 - bz0);
            const T mp = ev.at(-ax0 + bx0, -ay0 + by0, -az0 + bz0);
            const T mm = ev.at(-ax0 - bx0, -ay0 - by0, -az0 - bz0);
            const T h = (((pp - pm) - mp) + mm) * T(0.25);
            H[a][b] = h;
            H[b][a] = h;
        });
    });
}

// Derivative rule for moment fields along one axis (Sec. 3.5, last paragraph): central
// difference between fluid neighbours, second-order one-sided into the fluid next to a solid,
// first order with a single fluid neighbour on that side, zero with none.
// v[k] holds the field at offsets -2..2 (index k+2); fl[k] the fluid flags.
template <typename T>
__device__ __forceinline__ T deriv_rule(const T v[5], const bool fl[5]) {
    if (fl[3] && fl[1]) return (v[3] - v[1]) * T(0.5);
    if (fl[3]) return fl[4] ? ((T(-3) * v[2] + T(4) * v[3]) - v[4]) * T(0.5) : v[3] - v[2];
    if (fl[1]) return fl[0] ? ((T(3) * v[2] - T(4) * v[1]) + v[0]) * T(0.5) : v[2] - v[1];
    return T(0);
}

// Moment fields are stored packed per cell, (rho, w_x, w_y, w_z) in one 16-byte (FP32) or
// 32-byte (FP64) record, so a stencil neighbour costs one vector load plus its porosity.
template <typename T>
struct Packed;
template <>
struct Packed<float> {
    using type = float4;
};
template <>
struct Packed<double> {
    using type = double4;
};
template <typename T>
using P4 = typename Packed<T>::type;

template <typename T>
__device__ __forceinline__ P4<T> pack(T r, T a, T b, T c) {
    P4<T> q;
    q.x = r;
    q.y = a;
    q.z = b;
    q.w = c;
    return q;
}

// Moment record of one cell: intrinsic density, porosity, velocity.
template <typename T>
struct Rec {
    T r, e, w[3];
};

template <int D, typename T>
__device__ __forceinline__ Rec<T> load_rec(const P4<T> *__restrict__ m, uint32_t idx, T e) {
    const P4<T> q4 = ld(m, idx);
    Rec<T> q;
    q.r = q4.x;
    q.w[0] = q4.y;
    q.w[1] = q4.z;
    q.w[2] = q4.w;
    q.e = e;
    return q;
}

// m_b = rho w_b / eps of a record (the argument of Delta_nu in eqs. v_final and accel).
template <int D, typename T>
__device__ __forceinline__ void rec_m(const Rec<T> &q, T m[3]) {
#pragma unroll
    for (int b = 0; b < D; ++b) m[b] = dv(q.r * q.w[b], q.e);
}

// Load the axis neighbours of the cell with their fluid flags.
template <int D, typename T, bool SOLIDS, typename E>
__device__ __forceinline__ void load_stencil(const P4<T> *__restrict__ mom, const E &ev,
                                             const uint8_t *__restrict__ mask, const Grid &g,
                                             const Nbr<D> &nb, Rec<T> rec[3][2], bool fl[3][2]) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int k = s ? 1 : -1;
            const uint32_t m = nb.axis(g, a, k);
            rec[a][s] = load_rec<D>(mom, m, ev.at(a == 0 ? k : 0, a == 1 ? k : 0, a == 2 ? k : 0));
            fl[a][s] = SOLIDS ? !mask[m] : true;
        }
    }
}

// Variable-porosity viscous correction Delta_nu(m) at the cell, m = rho w / eps built from the
// records, eq. (porosity_correction_expanded):
//   nu {[H + tr(H) I] m + (div m) grad eps + (grad m) grad eps}
//     + nu' [|grad eps|^2 m + (m . grad eps) grad eps],   [(grad m) grad eps]_a = sum_b d_b m_a d_b eps.
template <int D, typename T, bool SOLIDS>
__device__ __forceinline__ void delta_nu(const P4<T> *__restrict__ mom,
                                         const T *__restrict__ eps,
                                         const uint8_t *__restrict__ mask, const Grid &g,
                                         const Nbr<D> &nb, const Rec<T> &own,
                                         const Rec<T> rec[3][2], const bool fl[3][2],
                                         const T ge[3], const T H[3][3], const Visc<T> &vs,
                                         T out[3]) {
    T mo[3];
    rec_m<D>(own, mo);
    T J[3][3];  // J[b][a] = d_a m_b
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T mm[3], mp[3];
        rec_m<D>(rec[a][0], mm);
        rec_m<D>(rec[a][1], mp);
        if (!SOLIDS || (fl[a][0] && fl[a][1])) {
#pragma unroll
            for (int b = 0; b < D; ++b) J[b][a] = (mp[b] - mm[b]) * T(0.5);
        } else {
            bool f5[5] = {false, fl[a][0], true, fl[a][1], false};
            T m2m[3] = {T(0), T(0), T(0)}, m2p[3] = {T(0), T(0), T(0)};
            if (fl[a][1] && !fl[a][0]) {
                const uint32_t p2 = nb.axis(g, a, 2);
                f5[4] = !mask[p2];
                if (f5[4]) rec_m<D>(load_rec<D>(mom, p2, ld(eps, p2)), m2p);
            }
            if (fl[a][0] && !fl[a][1]) {
                const uint32_t m2 = nb.axis(g, a, -2);
                f5[0] = !mask[m2];
                if (f5[0]) rec_m<D>(load_rec<D>(mom, m2, ld(eps, m2)), m2m);
            }
#pragma unroll
            for (int b = 0; b < D; ++b) {
                const T v5[5] = {m2m[b], mm[b], mo[b], mp[b], m2p[b]};
                J[b][a] = deriv_rule(v5, f5);
            }
        }
    }
    T trH = T(0), div = T(0), g2 = T(0), mg = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) trH = trH + H[a][a];
#pragma unroll
    for (int a = 0; a < D; ++a) div = div + J[a][a];
#pragma unroll
    for (int a = 0; a < D; ++a) g2 = g2 + ge[a] * ge[a];
#pragma unroll
    for (int a = 0; a < D; ++a) mg = mg + mo[a] * ge[a];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T Hm = T(0), Jg = T(0);
#pragma unroll
        for (int b = 0; b < D; ++b) Hm = Hm + H[a][b] * mo[b];
#pragma unroll
        for (int b = 0; b < D; ++b) Jg = Jg + J[a][b] * ge[b];
        const T t1 = Hm + trH * mo[a];
        const T t2 = div * ge[a];
        const T t3 = Jg;
        const T t4 = g2 * mo[a];
        const T t5 = mg * ge[a];
        out[a] = vs.nu * ((t1 + t2) + t3) + vs.dnu * (t4 + t5);
    }
}

// Derivative along axis a of a scalar built from a record (Phi^ext's flux, or v_a).
template <int D, typename T, bool SOLIDS, typename F>
__device__ __forceinline__ T record_deriv(const P4<T> *__restrict__ mom,
                                          const T *__restrict__ eps,
                                          const uint8_t *__restrict__ mask, const Grid &g,
                                          const Nbr<D> &nb, int a, const Rec<T> &own,
                                          const Rec<T> rec[3][2], const bool fl[3][2], F fn) {
    const T vm = fn(rec[a][0]), vp = fn(rec[a][1]);
    if (!SOLIDS || (fl[a][0] && fl[a][1])) return (vp - vm) * T(0.5);
    bool f5[5] = {false, fl[a][0], true, fl[a][1], false};
    T v5[5] = {T(0), vm, fn(own), vp, T(0)};
    if (fl[a][1] && !fl[a][0]) {
        const uint32_t p2 = nb.axis(g, a, 2);
        f5[4] = !mask[p2];
        if (f5[4]) v5[4] = fn(load_rec<D>(mom, p2, ld(eps, p2)));
    }
    if (fl[a][0] && !fl[a][1]) {
        const uint32_t m2 = nb.axis(g, a, -2);
        f5[0] = !mask[m2];
        if (f5[0]) v5[0] = fn(load_rec<D>(mom, m2, ld(eps, m2)));
    }
    return deriv_rule(v5, f5);
}

// Acceleration (accel) with Delta_nu(rho v / eps) from the record stencil (porosity_correction).
template <int D, typename T, bool SOLIDS>
__device__ __forceinline__ void accel_of(const P4<T> *__restrict__ mom,
                                         const T *__restrict__ eps, const T *__restrict__ muD,
                                         const T *__restrict__ muF,
                                         const uint8_t *__restrict__ mask, const Grid &g,
                                         const Phys<T> &ph, const Nbr<D> &nb, const Rec<T> &own,
                                         const Rec<T> rec[3][2], const bool fl[3][2],
                                         const T ge[3], const T H[3][3], const Visc<T> &vs,
                                         T acc[3]) {
    const uint32_t n = nb.self();
    T dm[3] = {T(0), T(0), T(0)};
    delta_nu<D, T, SOLIDS>(mom, eps, mask, g, nb, own, rec, fl, ge, H, vs, dm);
    T s = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) s = s + own.w[a] * own.w[a];
    const T vm = sq(s);
    const T md = ld(muD, n), mf = ld(muF, n);
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a)
        acc[a] = (((own.e * ph.b[a] - md * own.w[a]) - (mf * vm) * own.w[a]) + ph.RT * ge[a]) +
                 dv(dm[a], own.r);
}

// Equilibrium and shifted-equilibrium arguments of one cell from the moment fields (rho, v):
// acceleration (accel), Phi^ext (ex_corr), Phi^eta (eta_corr), then xi, P (xi_alpha_eq,
// P_alpha_alpha_eq) and xi*, P* (xi_alpha_*, P_aa_*) with lambda = 1.  `own` is the cell's
// record and rec / fl its axis neighbours; `mom` (the same step's records, or the previous
// step's in the lagged scheme) is read only for the one-sided stencils next to solids.
template <int D, typename T, bool SOLIDS, typename E>
__device__ __forceinline__ void forcing_args_stencil(
    const P4<T> *__restrict__ mom, const E &ev, const T *__restrict__ eps,
    const T *__restrict__ muD, const T *__restrict__ muF, const uint8_t *__restrict__ mask,
    const Grid &g, const Phys<T> &ph, const Nbr<D> &nb, const Rec<T> &own,
    const Rec<T> rec[3][2], const bool fl[3][2], const T ge[3], const T H[3][3],
    const Visc<T> &vs, T xi[3], T P[3], T xs[3], T Ps[3]) {
    T acc[3];
    accel_of<D, T, SOLIDS>(mom, eps, muD, muF, mask, g, ph, nb, own, rec, fl, ge, H, vs, acc);
    T phx[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T omr = ph.omr;
        auto gext = [a, omr](const Rec<T> &q) {
            const T va = q.w[a];
            return (q.r * va) * omr - dv(q.r * ((va * va) * va), q.e * q.e);
        };
        phx[a] = record_deriv<D, T, SOLIDS>(mom, eps, mask, g, nb, a, own, rec, fl, gext);
    }
    T pheta = T(0);
    if (ph.eta_on) {
        T divv = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            auto va = [a](const Rec<T> &q) { return q.w[a]; };
            divv = divv + record_deriv<D, T, SOLIDS>(mom, eps, mask, g, nb, a, own, rec, fl, va);
        }
        pheta = ((own.r * ph.RT) * (ph.two_over_D - dv(ph.eta, vs.nu))) * divv;
    }
    const T ier = dv(T(1), own.e * own.r);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xi[a] = dv(own.w[a], own.e);
        P[a] = xi[a] * xi[a] + ph.RT;
        xs[a] = dv(own.w[a] + acc[a], own.e);
        Ps[a] = (xs[a] * xs[a] + ph.RT) + ier * (phx[a] + pheta);
    }
}

// The same with the axis neighbours read from the records `mom`.
template <int D, typename T, bool SOLIDS, typename E>
__device__ __forceinline__ void forcing_args(const P4<T> *__restrict__ mom, const E &ev,
                                             const T *__restrict__ eps,
                                             const T *__restrict__ muD,
                                             const T *__restrict__ muF,
                                             const uint8_t *__restrict__ mask, const Grid &g,
                                             const Phys<T> &ph, const Nbr<D> &nb,
                                             const Rec<T> &own, const T ge[3], const T H[3][3],
                                             const Visc<T> &vs, T xi[3], T P[3], T xs[3],
                                             T Ps[3]) {
    Rec<T> rec[3][2];
    bool fl[3][2];
    load_stencil<D, T, SOLIDS>(mom, ev, mask, g, nb, rec, fl);
    forcing_args_stencil<D, T, SOLIDS>(mom, ev, eps, muD, muF, mask, g, ph, nb, own, rec, fl, ge,
                                       H, vs, xi, P, xs, Ps);
}

// One-dimensional factors of eq. (1d_scaled_eq) for c = -1, 0, +1.
template <typename T>
__device__ __forceinline__ void psi3(T xi, T P, T out[3]) {
    out[0] = (P - xi) * T(0.5);
    out[1] = T(1) - P;
    out[2] = (P + xi) * T(0.5);
}

// Products eps rho Psi_x Psi_y (Psi_z) of eq. (prod_form), taken in axis order; the partial
// products over (c_x, c_y) are shared by all c_z.
template <int D, typename T>
struct ProductForm {
    T pxy[3][3];
    T pz[3];
    __device__ __forceinline__ void init(T er, const T xi[3], const T P[3]) {
        T px[3], py[3];
        psi3(xi[0], P[0], px);
        psi3(xi[1], P[1], py);
        if constexpr (D == 3) psi3(xi[2], P[2], pz);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) pxy[i][j] = (er * px[i]) * py[j];
    }
    template <int I>
    __device__ __forceinline__ T at() const {
        using L = Lat<D>;
        constexpr int cx = L::c[I][0] + 1, cy = L::c[I][1] + 1, cz = L::c[I][2] + 1;
        if constexpr (D == 3) return pxy[cx][cy] * pz[cz];
        else return pxy[cx][cy];
    }
};

// Porosity record, derivatives and viscosity of the cell, the common prologue of the passes
// that work on the moment records.
template <int D, typename T>
struct CellStatic {
    T ge[3], H[3][3];
    Visc<T> vs;
};

template <int D, bool AD, typename T, typename E>
__device__ __forceinline__ CellStatic<D, T> cell_static(const E &ev, const Phys<T> &ph,
                                                        uint32_t n, T e0) {
    CellStatic<D, T> c;
    porosity_derivatives<D, AD>(ev, ph, n, e0, c.ge, c.H);
    c.vs = viscosity(ph, e0);
    return c;
}

// Where eps is locally uniform (zero gradient and Hessian: free fluid, or the plateau of a
// porous region) every term of Delta_nu carries a factor of them and vanishes.
template <int D, typename T>
__device__ __forceinline__ bool porosity_flat(const CellStatic<D, T> &cs) {
    bool flat = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        flat = flat && cs.ge[a] == T(0);
#pragma unroll
        for (int b = 0; b < D; ++b) flat = flat && cs.H[a][b] == T(0);
    }
    return flat;
}

// Velocity correction (v_final) from the cell's record and its axis neighbours rec / fl:
// v = v^(1) + Delta_nu(rho v^(1) / eps) / (2 rho); on flat porosity v = v^(1) + 0 (the value of
// the full evaluation) and the stencil is not used.
template <int D, typename T, bool SOLIDS>
__device__ __forceinline__ void velocity_from_stencil(const P4<T> *__restrict__ m1,
                                                      const T *__restrict__ eps,
                                                      const uint8_t *__restrict__ mask,
                                                      const Grid &g, const Nbr<D> &nb,
                                                      const Rec<T> &own, const Rec<T> rec[3][2],
                                                      const bool fl[3][2],
                                                      const CellStatic<D, T> &cs, bool flat,
                                                      T v[3]) {
    T dn[3] = {T(0), T(0), T(0)};
    if (!flat) delta_nu<D, T, SOLIDS>(m1, eps, mask, g, nb, own, rec, fl, cs.ge, cs.H, cs.vs, dn);
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = own.w[a] + dv(dn[a], T(2) * own.r);
}

// Velocity correction (v_final) from the cell's own record (rho, v^(1)) and the neighbour
// records in `m1`, read only where the porosity is not flat.
template <int D, typename T, bool SOLIDS, typename E>
__device__ __forceinline__ void corrected_velocity(const P4<T> *__restrict__ m1, const E &ev,
                                                   const T *__restrict__ eps,
                                                   const uint8_t *__restrict__ mask,
                                                   const Grid &g, const Nbr<D> &nb,
                                                   const Rec<T> &own, const CellStatic<D, T> &cs,
                                                   T v[3]) {
    const bool flat = porosity_flat<D, T>(cs);
    Rec<T> rec[3][2];
    bool fl[3][2];
    if (!flat) load_stencil<D, T, SOLIDS>(m1, ev, mask, g, nb, rec, fl);
    velocity_from_stencil<D, T, SOLIDS>(m1, eps, mask, g, nb, own, rec, fl, cs, flat, v);
}

// Equilibria of the cell (prod_form) for the equilibrium and shifted-equilibrium arguments.
template <int D, typename T, bool SOLIDS, typename E>
__device__ __forceinline__ void cell_equilibria(const P4<T> *__restrict__ m2, const E &ev,
                                                const T *__restrict__ eps,
                                                const T *__restrict__ muD,
                                                const T *__restrict__ muF,
                                                const uint8_t *__restrict__ mask, const Grid &g,
                                                const Phys<T> &ph, const Nbr<D> &nb,
                                                const Rec<T> &own, const CellStatic<D, T> &cs,
                                                ProductForm<D, T> &peq, ProductForm<D, T> &pst) {
    T xi[3], P[3], xs[3], Ps[3];
    forcing_args<D, T, SOLIDS>(m2, ev, eps, muD, muF, mask, g, ph, nb, own, cs.ge, cs.H, cs.vs,
                               xi, P, xs, Ps);
    const T er = own.e * own.r;
    peq.init(er, xi, P);
    pst.init(er, xs, Ps);
}

// ------------------------------------------------------------------------------------------
// Kernels, one thread per cell.  A workgroup of 256 threads owns a tx x ty x 1 tile
// (tx * ty = 256, tx = 256 for rows of 192 cells or more, so that the x-shifted accesses of the
// swapped AA phase stay inside one workgroup), or, with packed rows, 256 consecutive cells of a
// plane (see Tiling::packed).  Tiles are ordered so that stencil neighbours
// are processed close in time on the same XCD: the (tile-row, plane) grid is cut into blocks of
// by x bz tile rows, each block is traversed x-fastest then y then z, the blocks y-fastest then
// z, and the eight XCDs take contiguous ranges of that order (workgroup w runs on XCD w mod 8).
// A neighbour row in y or z is then at most by tiles away inside a block, and the shared L2 of
// the XCD still holds it.  Launch: block 256, grid 8 * per workgroups, per = ceil(tiles / 8).
// ------------------------------------------------------------------------------------------
struct Tiling {
    int tx, ty;       // tile shape, tx * ty = 256
    int ltx;          // log2(tx)
    int ntx, nty, ntz;
    int by, bz;       // block of tile rows
    int nby, nbz;     // blocks along y and z
    uint32_t per;     // tiles per XCD (padded order)
    // Packed rows (x extent not a multiple of 64, no LDS staging): a tile is 256 consecutive
    // cells of one z-plane in x-fastest order, wrapping from row to row, so that no wave is
    // left partly idle at the end of every row; "tile rows" are then these chunks.
    int packed;
    uint32_t pn;      // cells per plane, nx * ny
    uint64_t mnx;     // ceil(2^64 / nx): p / nx = umulhi64(p, mnx) for p < 2^32, nx >= 2
};

// Cell of this thread in tile w: returns -1 when the whole tile lies outside the order (the
// same for every thread of the workgroup), 0 when the thread's cell is outside the grid (ragged
// edge), 1 otherwise; (x0, y0) is the tile origin.
__device__ __forceinline__ int tile_cell(const Grid &g, const Tiling &tl, uint32_t w, int &x,
                                         int &y, int &z, int &x0, int &y0) {
    const uint32_t t = (w & 7u) * tl.per + (w >> 3);
    const uint32_t rows_per_block = (uint32_t)tl.by * (uint32_t)tl.bz;
    const uint32_t nt = (uint32_t)tl.ntx * rows_per_block * (uint32_t)tl.nby * (uint32_t)tl.nbz;
    if (t >= nt) return -1;
    const uint32_t tx = t % (uint32_t)tl.ntx;
    const uint32_t r = t / (uint32_t)tl.ntx;
    const uint32_t blk = r / rows_per_block, in = r % rows_per_block;
    const uint32_t ty = (blk % (uint32_t)tl.nby) * (uint32_t)tl.by + in % (uint32_t)tl.by;
    const uint32_t tz = (blk / (uint32_t)tl.nby) * (uint32_t)tl.bz + in / (uint32_t)tl.by;
    if (tl.packed) {
        if (ty >= (uint32_t)tl.nty || tz >= (uint32_t)g.nz) return -1;  // partial block
        const uint32_t p = ty * 256u + threadIdx.x;
        x0 = y0 = 0;
        z = (int)tz;
        if (p >= tl.pn) return 0;
        const uint32_t q = g.nx > 1 ? (uint32_t)__umul64hi((uint64_t)p, tl.mnx) : p;
        y = (int)q;
        x = (int)(p - q * (uint32_t)g.nx);
        return 1;
    }
    x0 = (int)(tx * (uint32_t)tl.tx);
    y0 = (int)(ty * (uint32_t)tl.ty);
    z = (int)tz;
    if (y0 >= g.ny || z >= g.nz) return -1;  // padding of a partial block
    x = x0 + (int)(threadIdx.x & (uint32_t)(tl.tx - 1));
    y = y0 + (int)(threadIdx.x >> (uint32_t)tl.ltx);
    return x < g.nx && y < g.ny ? 1 : 0;
}

// Cell prologue of the kernels that read porosity from global memory.
#define LBM_CELL_PROLOGUE_W(D, W)                                    \
    int x, y, z, x0_, y0_;                                           \
    if (tile_cell(g, tl, W, x, y, z, x0_, y0_) != 1) return;         \
    Nbr<D> nb;                                                       \
    nb.init(g, x, y, z);                                             \
    const uint32_t n = nb.self();                                    \
    const EpsGlobal<D, T> ev{eps, &nb};
#define LBM_CELL_PROLOGUE(D) LBM_CELL_PROLOGUE_W(D, blockIdx.x)

template <int D, bool STAGE, typename T>
__device__ __forceinline__ auto make_eps_view(const T *eps, const Nbr<D> *nb, const T *lds, int lx,
                                              int ly, const Tiling &tl) {
    if constexpr (STAGE) {
        const int row = tl.tx + 2, plane = row * (tl.ty + 2);
        return EpsTile<D, T>{lds + (D == 3 ? plane : 0) + (ly + 1) * row + lx + 1, row, plane};
    }
    else return EpsGlobal<D, T>{eps, nb};
}

// Prologue of the tiled passes.  With STAGE the workgroup first stages the porosity of its
// tile and halo in LDS (all threads, then a barrier) and threads outside the grid leave after
// it.  Staging pays where a cell reads the porosity of all its neighbours (the porous shift of
// 16-bit storage); where it reads only the derivative stencil, the barrier's exposed latency
// costs more than the gathers it saves (measured on the two-pass FP32 kernels).
#define LBM_TILE_PROLOGUE(D, W, STAGE)                               \
    int x, y, z, x0_, y0_;                                           \
    const int act_ = tile_cell(g, tl, W, x, y, z, x0_, y0_);         \
    if (act_ < 0) return;                                            \
    __shared__ T eps_lds_[(STAGE) ? EpsTile<D, T>::kSize : 1];       \
    if constexpr (STAGE) {                                           \
        stage_eps<D>(eps, g, tl.tx, tl.ty, x0_, y0_, z, eps_lds_);   \
        __syncthreads();                                             \
    }                                                                \
    if (!act_) return;                                               \
    Nbr<D> nb;                                                       \
    nb.init(g, x, y, z);                                             \
    const uint32_t n = nb.self();                                    \
    const auto ev = make_eps_view<D, (STAGE)>(eps, &nb, eps_lds_, x - x0_, y - y0_, tl);

// Density (transformed_density_moment), transformed momentum (transformed_momentum_moment),
// v^(0) (v_(0)) and the closed-form drag solve v^(1) (v_(1), velocity_coefficients) of a cell
// from its populations fi: returns the record (rho, eps, v^(1)).
template <int D, bool AD, typename T, typename E>
__device__ __forceinline__ Rec<T> cell_moments(const T fi[], const E &ev,
                                               const T *__restrict__ muD,
                                               const T *__restrict__ muF, const Nbr<D> &nb,
                                               const Phys<T> &ph, T *v0_out = nullptr) {
    using L = Lat<D>;
    const uint32_t n = nb.self();
    T S = T(0), Pi[3] = {T(0), T(0), T(0)};
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        S = S + fi[i];
        unroll<0, D>([&](auto ia) {
            constexpr int a = decltype(ia)::value;
            if constexpr (L::c[i][a] == 1) Pi[a] = Pi[a] + fi[i];
            else if constexpr (L::c[i][a] == -1) Pi[a] = Pi[a] - fi[i];
        });
    });
    const T e = ev.at(0, 0, 0);
    const T rho = div_rn(S, e);
    T v0[3];
    unroll<0, D>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        const T ge = eps_gradient<a, AD>(ev, ph, n);
        v0[a] = dv(Pi[a], rho) + T(0.5) * (e * ph.b[a] + ph.RT * ge);
    });
    const T c1 = T(1) + T(0.5) * ld(muD, n);
    const T c2 = T(0.5) * ld(muF, n);
    T s = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) s = s + v0[a] * v0[a];
    const T vm = sq(s);
    const T den = c1 + sq(c1 * c1 + (T(4) * c2) * vm);
    Rec<T> q;
    q.r = rho;
    q.e = e;
#pragma unroll
    for (int a = 0; a < 3; ++a) q.w[a] = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) q.w[a] = dv(T(2) * v0[a], den);
    if (v0_out) {
#pragma unroll
        for (int a = 0; a < 3; ++a) v0_out[a] = a < D ? v0[a] : T(0);
    }
    return q;
}

template <int D, typename T>
__device__ __forceinline__ void store_rec(P4<T> *__restrict__ m, uint32_t n, T r, const T w[3]) {
    *at(m, n) = pack(r, w[0], w[1], D == 3 ? w[2] : T(0));
}

// Groups of directions that can be loaded, collided and stored one after the other in place:
// the AA pattern writes a population into the slot its opposite is read from (in both phases,
// and for bounce-back), so each group holds whole opposite pairs.  D3Q27: [0, 9), [9, 19),
// [19, 27) (opposites are adjacent, from 1 on); D2Q9: one group.
template <int D>
struct PairGroups;
template <>
struct PairGroups<2> {
    static constexpr int n = 1;
    static constexpr int begin(int k) { return k == 0 ? 0 : 9; }
};
template <>
struct PairGroups<3> {
    static constexpr int n = 3;
    static constexpr int begin(int k) { return k == 0 ? 0 : (k == 1 ? 9 : (k == 2 ? 19 : 27)); }
};

// Collision (dicrete_scheme, momentum_rate with lambda = dt = 1) and streaming with halfway
// bounce-back, in place: f^pc_i = f_i + 2 beta (f^eq_i - f_i) + (1 - beta)(f^*_i - f^eq_i).
template <int D, typename T, typename P, bool SOLIDS, int PH>
__device__ __forceinline__ void collide_stream(P *__restrict__ f,
                                               const uint8_t *__restrict__ mask, const Grid &g,
                                               const Nbr<D> &nb, const T fi[], T beta, float base,
                                               const ProductForm<D, T> &peq,
                                               const ProductForm<D, T> &pst) {
    using L = Lat<D>;
    const T two_beta = T(2) * beta;
    const T omb = T(1) - beta;
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const T feq = peq.template at<i>();
        const T fst = pst.template at<i>();
        const T fpc = (fi[i] + two_beta * (feq - fi[i])) + omb * (fst - feq);
        store_pop<D, SOLIDS, PH, i>(f, mask, g, nb, fpc, base);
    });
}

// Pass one of the two-pass scheme: the record (rho, v^(1)) of every cell.  STAGE: the porosity
// of the tile and its halo is staged in LDS (16-bit storage on rectangular tiles).
template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD, bool STAGE>
__device__ __forceinline__ void moments_body_s(const P *__restrict__ f,
                                                 const T *__restrict__ eps,
                                                 const T *__restrict__ muD,
                                                 const T *__restrict__ muF,
                                                 const uint8_t *__restrict__ mask,
                                                 P4<T> *__restrict__ m1_out,
                                                 P4<T> *__restrict__ m0_out, Grid g, Tiling tl,
                                                 Phys<T> ph, uint32_t wg) {
    LBM_TILE_PROLOGUE(D, wg, (STAGE))
    using L = Lat<D>;
    if constexpr (SOLIDS) {
        if (mask[n]) {
            *at(m1_out, n) = pack(T(0), T(0), T(0), T(0));
            return;
        }
    }
    T fi[L::Q];
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        fi[i] = load_pop<D, SOLIDS, PH, i>(f, mask, ev, ph, g, nb);
    });
    T v0[3];
    const Rec<T> q = cell_moments<D, AD>(fi, ev, muD, muF, nb, ph, m0_out ? v0 : nullptr);
    store_rec<D>(m1_out, n, q.r, q.w);
    if (m0_out) store_rec<D>(m0_out, n, q.r, v0);  // base predictor for the Picard iterations
}

// Velocity correction (v_final) of every cell: reads the cell's own (rho, v^(1)) record from
// `own_src` and the neighbour records from `m1` (the same buffer in the two-pass scheme; the
// previous step's records when the lagged scheme reports moments), writes (rho, v).
template <int D, typename T, bool SOLIDS, bool AD>
__device__ __forceinline__ void vcorrect_body(const P4<T> *__restrict__ own_src,
                                                  const P4<T> *__restrict__ m1,
                                                  const T *__restrict__ eps,
                                                  const uint8_t *__restrict__ mask,
                                                  P4<T> *__restrict__ m2_out, Grid g, Tiling tl,
                                                  Phys<T> ph, uint32_t wg) {
    LBM_TILE_PROLOGUE(D, wg, (false))
    if constexpr (SOLIDS) {
        if (mask[n]) {
            *at(m2_out, n) = pack(T(0), T(0), T(0), T(0));
            return;
        }
    }
    const Rec<T> own = load_rec<D>(own_src, n, ev.at(0, 0, 0));
    const CellStatic<D, T> cs = cell_static<D, AD>(ev, ph, n, own.e);
    T v[3];
    corrected_velocity<D, T, SOLIDS>(m1, ev, eps, mask, g, nb, own, cs, v);
    store_rec<D>(m2_out, n, own.r, v);
}

// Loads of pair group K of a cell's populations in the arithmetic type (FP32 / FP64 storage).
template <int D, bool SOLIDS, int PH, int K, typename T, typename P, typename E>
__device__ __forceinline__ void load_pair_group(const P *__restrict__ f,
                                                const uint8_t *__restrict__ mask, const Grid &g,
                                                const Phys<T> &ph, const E &ev, const Nbr<D> &nb,
                                                T (&fa)[Lat<D>::Q]) {
    static_assert(!PopFmt<P>::shifted, "16-bit storage decodes after its loads");
    unroll<PairGroups<D>::begin(K), PairGroups<D>::begin(K + 1)>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        fa[i] = load_pop<D, SOLIDS, PH, i>(f, mask, ev, ph, g, nb);
    });
}

// Collision and streaming of the cell's populations with the equilibria peq, pst.  The
// populations are loaded only after the forcing arguments (FP32 / FP64 storage: except pair
// groups [0, FIRST), which the caller loaded into fa), in pair groups, so that fewer registers
// are live and more waves share each SIMD (16-bit storage: 3 -> 4 waves, 22 % faster).  With
// FP32 / FP64 storage the loads of group k + 1 are issued before the stores of group k, which
// can only reach slots that group k's own loads read (the AA pattern's slot of a population is
// read and written by the same cell, and a group holds whole opposite pairs): 256^3 box, FP32
// fused correction-collision kernel 0.885 -> 0.846 ms, FP64 2.05 -> 1.96 ms; the 16-bit forms
// load, decode, collide and store one group after the other (pipelined, their fused kernel
// spills: 0.75 -> 0.83 ms).
template <int D, typename T, typename P, bool SOLIDS, int PH, int FIRST = 0, typename E>
__device__ __forceinline__ void collide_populations(P *__restrict__ f,
                                                    const uint8_t *__restrict__ mask,
                                                    const Grid &g, const Phys<T> &ph,
                                                    const E &ev, const Nbr<D> &nb, T beta,
                                                    const ProductForm<D, T> &peq,
                                                    const ProductForm<D, T> &pst,
                                                    T (&fa)[Lat<D>::Q]) {
    static_assert(FIRST == 0 || !PopFmt<P>::shifted, "preloaded groups: FP32 / FP64 storage");
    __builtin_amdgcn_sched_barrier(0);
    const T two_beta = T(2) * beta;
    const T omb = T(1) - beta;
    const float base = own_base<P>(ev.at(0, 0, 0), ph);
    // Swapped phase: population addresses recomputed from an opaque copy of the neighbourhood
    // (16-bit storage 0.76 -> 0.68 ms on the 256^3 box, FP64 2 % faster).  FP32 storage keeps
    // the addresses of the stencil loads: 7 instead of 4 waves per SIMD left its collision as
    // fast as before, and the recomputation cost 1 %.
    constexpr bool kOpaque = PH == 1 && sizeof(P) != 4;
    const Nbr<D> nbp = kOpaque ? nb.opaque() : nb;
    auto collide_store = [&](auto gg) {
        constexpr int k = decltype(gg)::value;
        constexpr int g0 = PairGroups<D>::begin(k), g1 = PairGroups<D>::begin(k + 1);
        unroll<g0, g1>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const T feq = peq.template at<i>();
            const T fst = pst.template at<i>();
            const T fpc = (fa[i] + two_beta * (feq - fa[i])) + omb * (fst - feq);
            store_pop<D, SOLIDS, PH, i>(f, mask, g, nbp, fpc, base);
        });
    };
    if constexpr (PopFmt<P>::shifted) {
        unroll<0, PairGroups<D>::n>([&](auto gg) {
            constexpr int k = decltype(gg)::value;
            constexpr int g0 = PairGroups<D>::begin(k), g1 = PairGroups<D>::begin(k + 1);
            // Every load of the group is issued before the first decode.  With the decode next
            // to its load the scheduler kept one BF16 load in flight at a time (256^3 box:
            // BF16 collision 0.835 -> 0.601 ms, FP16 0.630 -> 0.601 ms; same results).
            P raw[g1 - g0];
            unroll<g0, g1>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                raw[i - g0] = load_raw<D, SOLIDS, PH, i>(f, mask, g, nbp);
            });
            __builtin_amdgcn_sched_barrier(0);
            T fi[g1 - g0];
            unroll<g0, g1>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                fi[i - g0] = decode<D, i, T>(raw[i - g0],
                                             load_sigma<D, SOLIDS, i, P>(mask, ev, ph, nbp));
            });
            unroll<g0, g1>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                const T feq = peq.template at<i>();
                const T fst = pst.template at<i>();
                const T fpc = (fi[i - g0] + two_beta * (feq - fi[i - g0])) + omb * (fst - feq);
                store_pop<D, SOLIDS, PH, i>(f, mask, g, nbp, fpc, base);
            });
            __builtin_amdgcn_sched_barrier(0);
        });
    } else {
        if constexpr (FIRST == 0)
            load_pair_group<D, SOLIDS, PH, 0>(f, mask, g, ph, ev, nbp, fa);
        unroll<0, PairGroups<D>::n>([&](auto gg) {
            constexpr int k = decltype(gg)::value;
            if constexpr (k + 1 < PairGroups<D>::n && k + 1 >= FIRST)
                load_pair_group<D, SOLIDS, PH, k + 1>(f, mask, g, ph, ev, nbp, fa);
            __builtin_amdgcn_sched_barrier(0);
            collide_store(gg);
            __builtin_amdgcn_sched_barrier(0);
        });
    }
}

template <int D, typename T, typename P, bool SOLIDS, int PH, typename E>
__device__ __forceinline__ void collide_populations(P *__restrict__ f,
                                                    const uint8_t *__restrict__ mask,
                                                    const Grid &g, const Phys<T> &ph,
                                                    const E &ev, const Nbr<D> &nb, T beta,
                                                    const ProductForm<D, T> &peq,
                                                    const ProductForm<D, T> &pst) {
    T fa[Lat<D>::Q];
    collide_populations<D, T, P, SOLIDS, PH, 0>(f, mask, g, ph, ev, nb, beta, peq, pst, fa);
}

// Pass two of the two-pass scheme: forcing from the (rho, v) records, collision, streaming.
// The cell's own record comes from m2 and its stencil neighbours' from nbr: the same buffer in
// the two-pass scheme, the previous step's records in a lagged step run as separate passes.
template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD>
__device__ __forceinline__ void collide_body(P *__restrict__ f,
                                                 const P4<T> *__restrict__ m2,
                                                 const P4<T> *__restrict__ nbr,
                                                 const T *__restrict__ eps,
                                                 const T *__restrict__ muD,
                                                 const T *__restrict__ muF,
                                                 const uint8_t *__restrict__ mask, Grid g,
                                                 Tiling tl, Phys<T> ph, uint32_t wg) {
    LBM_TILE_PROLOGUE(D, wg, (false))
    if constexpr (SOLIDS) {
        if (mask[n]) return;
    }
    const Rec<T> own = load_rec<D>(m2, n, ev.at(0, 0, 0));
    const CellStatic<D, T> cs = cell_static<D, AD>(ev, ph, n, own.e);
    ProductForm<D, T> peq, pst;
    cell_equilibria<D, T, SOLIDS>(nbr, ev, eps, muD, muF, mask, g, ph, nb, own, cs, peq, pst);
    collide_populations<D, T, P, SOLIDS, PH>(f, mask, g, ph, ev, nb, cs.vs.beta, peq, pst);
}

// One pass of the lagged scheme: the cell's own moments, velocity correction and forcing are
// those of the current populations, while the neighbour values entering Delta_nu, Phi^ext and
// Phi^eta are the previous step's records (m1p: rho, v^(1); m2p: rho, v).  The cell's new
// records go to m1n / m2n for the next step.  A steady state of this scheme is a steady state
// of the two-pass scheme.
template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD, bool STAGE>
__device__ __forceinline__ void fused_body_s(P *__restrict__ f, const P4<T> *__restrict__ m1p,
                                               const P4<T> *__restrict__ m2p,
                                               P4<T> *__restrict__ m1n, P4<T> *__restrict__ m2n,
                                               const T *__restrict__ eps,
                                               const T *__restrict__ muD,
                                               const T *__restrict__ muF,
                                               const uint8_t *__restrict__ mask, Grid g,
                                               Tiling tl, Phys<T> ph, uint32_t wg) {
    LBM_TILE_PROLOGUE(D, wg, (STAGE))
    using L = Lat<D>;
    if constexpr (SOLIDS) {
        if (mask[n]) {
            *at(m1n, n) = pack(T(0), T(0), T(0), T(0));
            *at(m2n, n) = pack(T(0), T(0), T(0), T(0));
            return;
        }
    }
    T fi[L::Q];
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        fi[i] = load_pop<D, SOLIDS, PH, i>(f, mask, ev, ph, g, nb);
    });
    const Rec<T> own1 = cell_moments<D, AD>(fi, ev, muD, muF, nb, ph);
    const CellStatic<D, T> cs = cell_static<D, AD>(ev, ph, n, own1.e);
    Rec<T> own2 = own1;
    corrected_velocity<D, T, SOLIDS>(m1p, ev, eps, mask, g, nb, own1, cs, own2.w);
    ProductForm<D, T> peq, pst;
    cell_equilibria<D, T, SOLIDS>(m2p, ev, eps, muD, muF, mask, g, ph, nb, own2, cs, peq, pst);
    collide_stream<D, T, P, SOLIDS, PH>(f, mask, g, PH == 1 ? nb.opaque() : nb, fi, cs.vs.beta,
                                        own_base<P>(ev.at(0, 0, 0), ph), peq, pst);
    store_rec<D>(m1n, n, own1.r, own1.w);
    store_rec<D>(m2n, n, own2.r, own2.w);
}

// One Picard iteration of the second-order velocity evaluation (App. F):
//   s = v_0 + Delta_nu(rho v^(k) / eps) / (2 rho),  v^(k+1) = 2 s / (c_1 + sqrt(c_1^2 + 4 c_2 |s|)),
// under-relaxed by omega when omega != 1; reads the (rho, v^(k)) records of the cell and its
// neighbours and the cell's (rho, v_0) record, writes (rho, v^(k+1)).
template <int D, typename T, bool SOLIDS, bool AD>
__device__ __forceinline__ void picard_body(const P4<T> *__restrict__ vin,
                                            const P4<T> *__restrict__ m0,
                                            const T *__restrict__ eps,
                                            const T *__restrict__ muD,
                                            const T *__restrict__ muF,
                                            const uint8_t *__restrict__ mask,
                                            P4<T> *__restrict__ vout, Grid g, Tiling tl,
                                            Phys<T> ph, T omega, uint32_t wg) {
    LBM_TILE_PROLOGUE(D, wg, false)
    if constexpr (SOLIDS) {
        if (mask[n]) {
            *at(vout, n) = pack(T(0), T(0), T(0), T(0));
            return;
        }
    }
    const Rec<T> own = load_rec<D>(vin, n, ev.at(0, 0, 0));
    const CellStatic<D, T> cs = cell_static<D, AD>(ev, ph, n, own.e);
    Rec<T> rec[3][2];
    bool fl[3][2];
    load_stencil<D, T, SOLIDS>(vin, ev, mask, g, nb, rec, fl);
    T dn[3];
    delta_nu<D, T, SOLIDS>(vin, eps, mask, g, nb, own, rec, fl, cs.ge, cs.H, cs.vs, dn);
    const P4<T> q0 = ld(m0, n);
    const T v0[3] = {q0.y, q0.z, q0.w};
    T sv[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) sv[a] = v0[a] + dv(dn[a], T(2) * own.r);
    const T c1 = T(1) + T(0.5) * ld(muD, n);
    const T c2 = T(0.5) * ld(muF, n);
    T s = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) s = s + sv[a] * sv[a];
    const T den = c1 + sq(c1 * c1 + (T(4) * c2) * sq(s));
    T v[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T vk = dv(T(2) * sv[a], den);
        v[a] = omega == T(1) ? vk : (T(1) - omega) * own.w[a] + omega * vk;
    }
    store_rec<D>(vout, n, own.r, v);
}

template <int D, typename T, bool SOLIDS, bool AD>
__global__ __launch_bounds__(256) void k_picard(const P4<T> *__restrict__ vin,
                                                const P4<T> *__restrict__ m0,
                                                const T *__restrict__ eps,
                                                const T *__restrict__ muD,
                                                const T *__restrict__ muF,
                                                const uint8_t *__restrict__ mask,
                                                P4<T> *__restrict__ vout, Grid g, Tiling tl,
                                                Phys<T> ph, T omega) {
    picard_body<D, T, SOLIDS, AD>(vin, m0, eps, muD, muF, mask, vout, g, tl, ph, omega, blockIdx.x);
}

// The moment and lagged passes of a tile: 16-bit storage stages the porosity its decode reads
// in LDS on rectangular tiles and reads it through the caches on packed rows (ragged x extents),
// whose tiles have no rectangular halo.  Same values either way.
template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD>
__device__ __forceinline__ void moments_body(const P *__restrict__ f, const T *__restrict__ eps,
                                             const T *__restrict__ muD, const T *__restrict__ muF,
                                             const uint8_t *__restrict__ mask,
                                             P4<T> *__restrict__ m1_out, P4<T> *__restrict__ m0_out,
                                             Grid g, Tiling tl, Phys<T> ph, uint32_t wg) {
    if constexpr (PopFmt<P>::shifted) {
        if (tl.packed) {
            moments_body_s<D, T, P, SOLIDS, PH, AD, false>(f, eps, muD, muF, mask, m1_out, m0_out,
                                                           g, tl, ph, wg);
            return;
        }
    }
    moments_body_s<D, T, P, SOLIDS, PH, AD, PopFmt<P>::shifted>(f, eps, muD, muF, mask, m1_out,
                                                                 m0_out, g, tl, ph, wg);
}

template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD>
__device__ __forceinline__ void fused_body(P *__restrict__ f, const P4<T> *__restrict__ m1p,
                                           const P4<T> *__restrict__ m2p, P4<T> *__restrict__ m1n,
                                           P4<T> *__restrict__ m2n, const T *__restrict__ eps,
                                           const T *__restrict__ muD, const T *__restrict__ muF,
                                           const uint8_t *__restrict__ mask, Grid g, Tiling tl,
                                           Phys<T> ph, uint32_t wg) {
    if constexpr (PopFmt<P>::shifted) {
        if (tl.packed) {
            fused_body_s<D, T, P, SOLIDS, PH, AD, false>(f, m1p, m2p, m1n, m2n, eps, muD, muF,
                                                         mask, g, tl, ph, wg);
            return;
        }
    }
    fused_body_s<D, T, P, SOLIDS, PH, AD, PopFmt<P>::shifted>(f, m1p, m2p, m1n, m2n, eps, muD,
                                                               muF, mask, g, tl, ph, wg);
}

// Single-run kernels: workgroup w handles tile w of the run.
//
// Runs with solid cells: the solid-aware code (mask checks on every stencil and streaming
// access) is needed only by tiles that have a solid cell within one cell (in any direction) of
// one of their cells; every other tile takes the solid-free code, which evaluates the same
// expressions.  tsolid[w] (k_tile_solid) tells which; null means every tile is solid-aware.
__device__ __forceinline__ bool tile_free(const uint8_t *__restrict__ tsolid) {
    return tsolid && !tsolid[blockIdx.x];
}

template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD>
__global__ __launch_bounds__(256) void k_moments(const P *__restrict__ f,
                                                 const T *__restrict__ eps,
                                                 const T *__restrict__ muD,
                                                 const T *__restrict__ muF,
                                                 const uint8_t *__restrict__ mask,
                                                 const uint8_t *__restrict__ tsolid,
                                                 P4<T> *__restrict__ m1_out,
                                                 P4<T> *__restrict__ m0_out, Grid g, Tiling tl,
                                                 Phys<T> ph) {
    if constexpr (SOLIDS) {
        if (tile_free(tsolid)) {
            moments_body<D, T, P, false, PH, AD>(f, eps, muD, muF, mask, m1_out, m0_out, g, tl,
                                                 ph, blockIdx.x);
            return;
        }
    }
    // FP32 storage without solids walks the tiles in their linear order rather than in one
    // range per XCD: all XCDs then stream neighbouring rows at once (256^3 box 0.445 -> 0.435
    // ms; FP64 and the 16-bit forms were 1-2 % slower so): workgroup w takes tile w, passed as
    // the index (w % per) * 8 + w / per that the XCD mapping of tile_cell sends to w.
    const uint32_t wt = !SOLIDS && std::is_same_v<P, float>
                            ? (blockIdx.x % tl.per) * 8u + blockIdx.x / tl.per
                            : blockIdx.x;
    moments_body<D, T, P, SOLIDS, PH, AD>(f, eps, muD, muF, mask, m1_out, m0_out, g, tl, ph, wt);
}

// Velocity correction of a tile whose every cell has a uniform porosity neighbourhood: Delta_nu
// vanishes, v = v^(1) + 0 (the value of the full evaluation), from the cell's own record only.
// A solid cell's record is zero (the moment pass writes it so), and so is its copy: no mask
// read is needed.
template <int D, typename T>
__device__ __forceinline__ void vcorrect_flat_body(const P4<T> *__restrict__ own_src,
                                                   P4<T> *__restrict__ m2_out, Grid g,
                                                   Tiling tl, uint32_t wg) {
    int x, y, z, x0_, y0_;
    if (tile_cell(g, tl, wg, x, y, z, x0_, y0_) != 1) return;
    const uint32_t n = (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
    const P4<T> q = ld(own_src, n);
    *at(m2_out, n) = pack(q.x, q.y + T(0), q.z + T(0), D == 3 ? q.w + T(0) : T(0));
}

template <int D, typename T, bool SOLIDS, bool AD>
__global__ __launch_bounds__(256) void k_vcorrect(const P4<T> *__restrict__ own_src,
                                                  const P4<T> *__restrict__ m1,
                                                  const T *__restrict__ eps,
                                                  const uint8_t *__restrict__ mask,
                                                  const uint8_t *__restrict__ tsolid,
                                                  const uint8_t *__restrict__ tflat,
                                                  P4<T> *__restrict__ m2_out, Grid g, Tiling tl,
                                                  Phys<T> ph) {
    // tflat[w] = 0: no cell of tile w has a porosity gradient or Hessian (k_tile_flat)
    if (tflat && !tflat[blockIdx.x]) {
        vcorrect_flat_body<D, T>(own_src, m2_out, g, tl, blockIdx.x);
        return;
    }
    if constexpr (SOLIDS) {
        if (tile_free(tsolid)) {
            vcorrect_body<D, T, false, AD>(own_src, m1, eps, mask, m2_out, g, tl, ph, blockIdx.x);
            return;
        }
    }
    vcorrect_body<D, T, SOLIDS, AD>(own_src, m1, eps, mask, m2_out, g, tl, ph, blockIdx.x);
}

// Waves per SIMD requested for the kernels of runs with solids.  Such a kernel holds the
// solid-free and the solid-aware code, and the latter, run only by tiles next to a solid, needs
// more registers; left alone it would set the occupancy of every tile.  Where it pays, the
// occupancy of the solid-free code is requested and the solid-aware code spills a few values
// instead (D3Q27 sphere duct, 768 x 384 x 384: 16-bit collision 5.24 -> 4.62 ms, 16-bit lagged
// pass 9.47 -> 8.29 ms, FP64 swapped-phase collision 12.13 -> 11.89 ms; the same for FP32 cost
// 2 %, so FP32 requests nothing).  That holds where few tiles are solid-aware (4 % in that
// duct); where most are (the pressure-driven duct's solid x faces make two of every row's three
// tiles solid-aware) the spills cost more than the occupancy gains (FP16 collision 12.70 ->
// 8.55 ms without the request), so the host launches the requesting instantiation (OCC) only
// for runs whose tiles are less than a quarter solid-aware.  1 requests nothing.
template <int D, typename T, typename P, bool SOLIDS, int PH, bool OCC = true>
struct SolidAwareWaves {
    static constexpr bool on = SOLIDS && D == 3 && OCC;
    static constexpr bool half = sizeof(P) == 2, fp64 = sizeof(T) == 8;
    static constexpr int collide = !on ? 1 : half ? (PH == 1 ? 5 : 6) : (fp64 && PH == 1 ? 3 : 1);
    static constexpr int fused = on && half && PH == 0 ? 3 : 1;
};

template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD, bool OCC>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(SolidAwareWaves<D, T, P, SOLIDS, PH, OCC>::collide)))
void k_collide(P *__restrict__ f, const P4<T> *__restrict__ m2, const P4<T> *__restrict__ nbr,
               const T *__restrict__ eps, const T *__restrict__ muD, const T *__restrict__ muF,
               const uint8_t *__restrict__ mask, const uint8_t *__restrict__ tsolid, Grid g,
               Tiling tl, Phys<T> ph) {
    if constexpr (SOLIDS) {
        if (tile_free(tsolid)) {
            collide_body<D, T, P, false, PH, AD>(f, m2, nbr, eps, muD, muF, mask, g, tl, ph,
                                                 blockIdx.x);
            return;
        }
    }
    collide_body<D, T, P, SOLIDS, PH, AD>(f, m2, nbr, eps, muD, muF, mask, g, tl, ph,
                                          blockIdx.x);
}

// ------------------------------------------------------------------------------------------
// Two-pass step with the velocity correction fused into the collision pass (D3Q27, no solids,
// differenced porosity derivatives; populations in the arithmetic type or shifted 16-bit, whose
// decode reads the porosity of each population's source cell from the staged planes).  The collision
// of a cell reads the corrected velocity of the cell and its six face neighbours, and the
// correction of a cell reads the (rho, v^(1)) records of its own six face neighbours.  A
// workgroup owns a tile of cells (ZCfg: 128 x 4 in FP32) and marches it through a chunk of
// z-planes.  Its first waves correct the velocity of the tile and its one-cell ring in x and y
// (776 cells at 128 x 4, from the records of the moment pass exactly as the separate
// correction pass reads them) two planes ahead, into a ring of four planes in LDS, while its
// other waves (one thread per tile cell) collide the current plane from the ring; one barrier
// per plane.  The corrected velocities never go through HBM (the separate pass writes them
// and the collision reads them back, 32 B per cell), at the price of correcting the ring cells
// (1.52x at 128 x 4) and the chunk's end planes again.  The correcting waves read their records and porosity from planes staged in
// LDS (loaded once per plane, coalesced, two planes ahead), and the colliding waves read their
// porosity there too.  256^3 box, FP32, per step: the separate passes 0.225 + 0.833 ms; 64 x 4
// tiles with four correcting and four colliding waves 1.045 ms (with three or two correcting
// waves 1.22 and 1.38 ms); 64 x 8 tiles 1.012 ms; staged correction inputs 0.959 ms; staged
// collision porosity 0.906 ms (chunks of 128 planes); the shapes and thread counts of ZCfg and
// the loads of collide_populations brought it to 0.815 ms.  Loading the next plane's first
// pair group before the barrier did not pay (0.824 -> 0.844 ms).
// With the two kinds of work in different waves, the correction's arithmetic and cached
// gathers run beside the collision's HBM streams instead of between them.  Every expression
// is the separate passes' own, so the results are bitwise the same.
struct ZTiling {
    int ntx, nty, nch;  // tiles along x (ZCfg::kX cells) and y (ZCfg::kY rows), chunks along z
    int zc;             // planes per chunk
    uint32_t per;       // workgroups per XCD (padded)
};
// Shape of a fused workgroup for arithmetic type T and population storage P: a kX x kY tile
// (kX * kY collision threads and kProd correcting threads), the ring of corrected velocities
// (kRX x kRY) and the staged region of the correcting waves (the tile and two rings,
// kSX x kSY).  FP32 takes 128 x 4 tiles: fewer tile edges in x, across which the swapped
// phase's x-shifted accesses reach lines that another workgroup loads and stores (256^3 box:
// 0.886 ms against 0.901 for 64 x 8, which corrects fewer ring cells); the 16-bit forms 64 x 8
// (0.747 ms against 0.780); FP64 64 x 4, as its LDS rings would not fit 160 KB otherwise.
// FP32 and the 16-bit forms correct with half as many threads as they collide with: 768
// threads per workgroup leave each thread up to 168 registers instead of 128, which ends the
// 16-bit collision's spills (FP16 0.763 -> 0.700 ms, FP32 0.828 -> 0.815 ms; a quarter as
// many correcting threads made the 16-bit kernel correction-bound, 1.08 ms).
template <typename T, typename P = T>
struct ZCfg {
    static constexpr bool kF64 = sizeof(T) == 8, kHalf = sizeof(P) == 2;
    static constexpr int kX = kF64 || kHalf ? 64 : 128, kY = kF64 ? 4 : (kHalf ? 8 : 4);
    static constexpr int kRX = kX + 2, kRY = kY + 2, kR = kRX * kRY;
    static constexpr int kSX = kX + 4, kSY = kY + 4, kS = kSX * kSY;
    static constexpr int kProd = kF64 ? kX * kY : kX * kY / 2, kThreads = kProd + kX * kY;
};

// Porosity of a cell's 3x3x3 neighbourhood from planes staged in LDS.
template <typename T>
struct EpsRing {
    const T *p[3];  // the cell's own entry in the planes z - 1, z, z + 1
    int row;
    __device__ __forceinline__ T at(int dx, int dy, int dz) const {
        return p[dz + 1][dy * row + dx];
    }
};

template <typename T, typename PS, int PH>
__global__ __launch_bounds__((ZCfg<T, PS>::kThreads)) void k_collide_vc(PS *__restrict__ f,
                                                          const P4<T> *__restrict__ m1,
                                                          const T *__restrict__ eps,
                                                          const T *__restrict__ muD,
                                                          const T *__restrict__ muF, Grid g,
                                                          ZTiling zt, Phys<T> ph) {
    constexpr int D = 3;
    using C = ZCfg<T, PS>;
    constexpr int kZX = C::kX, kZY = C::kY, kZRX = C::kRX, kZRY = C::kRY, kZR = C::kR;
    constexpr int kZSX = C::kSX, kZS = C::kS, kZProd = C::kProd;
    // (rho, v) of four consecutive planes on the tile and its ring: slot of plane z (z - z0 + 4) & 3
    __shared__ P4<T> vr[4][kZR];
    // (rho, v^(1)) records of four consecutive planes on the tile and two rings (kZSX x kZSY
    // cells), the correcting waves' inputs: slot of plane z (z - z0 + 8) & 3; porosity of six
    // (the colliding waves read the planes z - 1 .. z + 1 from it too): slot (z - z0 + 12) % 6
    __shared__ P4<T> rs[4][kZS];
    __shared__ T es[6][kZS];
    const uint32_t t = (blockIdx.x & 7u) * zt.per + (blockIdx.x >> 3);
    if (t >= (uint32_t)zt.ntx * (uint32_t)zt.nty * (uint32_t)zt.nch) return;  // whole workgroup
    const int x0 = (int)(t % (uint32_t)zt.ntx) * kZX;
    const uint32_t r = t / (uint32_t)zt.ntx;
    const int y0 = (int)(r % (uint32_t)zt.nty) * kZY;
    const int z0 = (int)(r / (uint32_t)zt.nty) * zt.zc;
    const int z1 = min(z0 + zt.zc, g.nz);
    // the first kZProd threads correct velocities, the others collide (the branch is uniform
    // per wave)
    const bool producer = threadIdx.x < (uint32_t)kZProd;
    const int tid = producer ? (int)threadIdx.x : (int)threadIdx.x - kZProd;
    auto wrap = [](int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); };
    auto vslot = [&](int zz) { return (zz - z0 + 4) & 3; };
    auto sslot = [&](int zz) { return (zz - z0 + 8) & 3; };
    auto eslot = [&](int zz) { return (zz - z0 + 12) % 6; };
    auto rec_at = [](const P4<T> &q, T e) {
        Rec<T> o;
        o.r = q.x;
        o.w[0] = q.y;
        o.w[1] = q.z;
        o.w[2] = q.w;
        o.e = e;
        return o;
    };

    // staging of plane zz (z0 - 2 <= zz <= z1 + 1): loads into registers, then LDS stores, so
    // that the loads of the next plane are in flight while the current one is corrected
    constexpr int kSt = (kZS + kZProd - 1) / kZProd;
    P4<T> sr[kSt];
    T se[kSt];
    auto stage_load = [&](int zz) {
        const int zp = wrap(zz, g.nz);
#pragma unroll
        for (int k = 0; k < kSt; ++k) {
            const int e = tid + k * kZProd;
            if (e < kZS) {
                const int sx = e % kZSX, sy = e / kZSX;
                const uint32_t c = (uint32_t)wrap(x0 - 2 + sx, g.nx) +
                                   (uint32_t)g.nx * ((uint32_t)wrap(y0 - 2 + sy, g.ny) +
                                                     (uint32_t)g.ny * (uint32_t)zp);
                sr[k] = ld(m1, c);
                se[k] = ld(eps, c);
            }
        }
    };
    auto stage_store = [&](int zz) {
        const int sl = sslot(zz), el = eslot(zz);
#pragma unroll
        for (int k = 0; k < kSt; ++k) {
            const int e = tid + k * kZProd;
            if (e < kZS) {
                rs[sl][e] = sr[k];
                es[el][e] = se[k];
            }
        }
    };
    // corrected velocity of plane zz (z0 - 1 <= zz <= z1) on the tile and its ring, from the
    // staged planes zz - 1, zz, zz + 1
    auto correct_plane = [&](int zz) {
        P4<T> *dst = vr[vslot(zz)];
        const P4<T> *rm = rs[sslot(zz - 1)], *rc = rs[sslot(zz)], *rp = rs[sslot(zz + 1)];
        for (int j = tid; j < kZR; j += kZProd) {
            const int rx = j % kZRX, ry = j / kZRX;
            if ((rx == 0 || rx == kZRX - 1) && (ry == 0 || ry == kZRY - 1)) continue;  // corners
            const int q = (ry + 1) * kZSX + rx + 1;  // the cell in the staged region
            const EpsRing<T> ev{{es[eslot(zz - 1)] + q, es[eslot(zz)] + q, es[eslot(zz + 1)] + q},
                                kZSX};
            const Rec<T> own = rec_at(rc[q], ev.at(0, 0, 0));
            const CellStatic<D, T> cs = cell_static<D, false>(ev, ph, 0u, own.e);
            const bool flat = porosity_flat<D, T>(cs);
            Rec<T> rec[3][2];
            bool fl[3][2];
            if (!flat) {
                rec[0][0] = rec_at(rc[q - 1], ev.at(-1, 0, 0));
                rec[0][1] = rec_at(rc[q + 1], ev.at(1, 0, 0));
                rec[1][0] = rec_at(rc[q - kZSX], ev.at(0, -1, 0));
                rec[1][1] = rec_at(rc[q + kZSX], ev.at(0, 1, 0));
                rec[2][0] = rec_at(rm[q], ev.at(0, 0, -1));
                rec[2][1] = rec_at(rp[q], ev.at(0, 0, 1));
#pragma unroll
                for (int a = 0; a < 3; ++a) fl[a][0] = fl[a][1] = true;
            }
            T v[3];
            const Nbr<D> none{};
            velocity_from_stencil<D, T, false>(nullptr, nullptr, nullptr, g, none, own, rec, fl,
                                               cs, flat, v);
            dst[j] = pack(own.r, v[0], v[1], v[2]);
        }
    };

    // prologue: planes z0 - 2 .. z0 + 1 staged, corrections of z0 - 1 and z0, then z0 + 2
    // staged and z0 + 1 corrected while z0 + 3 is loaded
    if (producer) {
        for (int zz = z0 - 2; zz <= z0 + 1; ++zz) {
            stage_load(zz);
            stage_store(zz);
        }
    }
    __syncthreads();
    if (producer) {
        stage_load(z0 + 2);
        correct_plane(z0 - 1);
        correct_plane(z0);
    }
    __syncthreads();
    if (producer) stage_store(z0 + 2);
    __syncthreads();
    if (producer) {
        stage_load(z0 + 3);
        correct_plane(z0 + 1);
        stage_store(z0 + 3);
    }
    __syncthreads();
    const int lx = tid % kZX, ly = tid / kZX;
    const int j = (ly + 1) * kZRX + lx + 1;
    for (int zz = z0; zz < z1; ++zz) {
        if (producer) {
            // the plane after next from the staged planes zz + 1 .. zz + 3, while plane zz + 4
            // is loaded into the slot of plane zz (which no correction reads any more)
            if (zz + 2 <= z1) {
                if (zz + 4 <= z1 + 1) stage_load(zz + 4);
                correct_plane(zz + 2);
                if (zz + 4 <= z1 + 1) stage_store(zz + 4);
            }
        } else {
            const P4<T> *vm = vr[vslot(zz - 1)], *vc = vr[vslot(zz)], *vp = vr[vslot(zz + 1)];
            Nbr<D> nb;
            nb.init(g, x0 + lx, y0 + ly, zz);
            const int qc = (ly + 2) * kZSX + lx + 2;  // the cell in the staged region
            const EpsRing<T> ev{{es[eslot(zz - 1)] + qc, es[eslot(zz)] + qc, es[eslot(zz + 1)] + qc},
                                kZSX};
            const uint32_t n = nb.self();
            // FP32 / FP64: the first pair group's loads are in flight during the forcing
            // (256^3 box, FP32 0.849 -> 0.822 ms, FP64 1.98 -> 1.89 ms)
            T fa[27];
            if constexpr (!PopFmt<PS>::shifted)
                load_pair_group<D, false, PH, 0>(f, nullptr, g, ph, ev, nb, fa);
            const Rec<T> own = rec_at(vc[j], ev.at(0, 0, 0));
            const CellStatic<D, T> cs = cell_static<D, false>(ev, ph, n, own.e);
            Rec<T> rec[3][2];
            bool fl[3][2];
            rec[0][0] = rec_at(vc[j - 1], ev.at(-1, 0, 0));
            rec[0][1] = rec_at(vc[j + 1], ev.at(1, 0, 0));
            rec[1][0] = rec_at(vc[j - kZRX], ev.at(0, -1, 0));
            rec[1][1] = rec_at(vc[j + kZRX], ev.at(0, 1, 0));
            rec[2][0] = rec_at(vm[j], ev.at(0, 0, -1));
            rec[2][1] = rec_at(vp[j], ev.at(0, 0, 1));
#pragma unroll
            for (int a = 0; a < 3; ++a) fl[a][0] = fl[a][1] = true;
            T xi[3], P[3], xs[3], Ps[3];
            forcing_args_stencil<D, T, false>(nullptr, ev, eps, muD, muF, nullptr, g, ph, nb, own,
                                              rec, fl, cs.ge, cs.H, cs.vs, xi, P, xs, Ps);
            ProductForm<D, T> peq, pst;
            const T er = own.e * own.r;
            peq.init(er, xi, P);
            pst.init(er, xs, Ps);
            collide_populations<D, T, PS, false, PH, (PopFmt<PS>::shifted ? 0 : 1)>(
                f, nullptr, g, ph, ev, nb, cs.vs.beta, peq, pst, fa);
        }
        __syncthreads();
    }
}

template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD, bool OCC>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(SolidAwareWaves<D, T, P, SOLIDS, PH, OCC>::fused)))
void k_fused(P *__restrict__ f, const P4<T> *__restrict__ m1p, const P4<T> *__restrict__ m2p,
             P4<T> *__restrict__ m1n, P4<T> *__restrict__ m2n, const T *__restrict__ eps,
             const T *__restrict__ muD, const T *__restrict__ muF,
             const uint8_t *__restrict__ mask, const uint8_t *__restrict__ tsolid, Grid g,
             Tiling tl, Phys<T> ph) {
    if constexpr (SOLIDS) {
        if (tile_free(tsolid)) {
            fused_body<D, T, P, false, PH, AD>(f, m1p, m2p, m1n, m2n, eps, muD, muF, mask, g, tl,
                                               ph, blockIdx.x);
            return;
        }
    }
    fused_body<D, T, P, SOLIDS, PH, AD>(f, m1p, m2p, m1n, m2n, eps, muD, muF, mask, g, tl, ph,
                                        blockIdx.x);
}

// tsolid[w] = 1 when a cell of tile w, or a cell within one cell of one of them (faces, edges
// and corners, through the periodic wrap), is solid.  Same grid and tile order as the passes;
// workgroups past the last tile write nothing (the passes return before reading theirs).
template <int D>
__global__ __launch_bounds__(256) void k_tile_solid(const uint8_t *__restrict__ mask, Grid g,
                                                    Tiling tl, uint8_t *__restrict__ tsolid) {
    int x, y, z, x0, y0;
    const int act = tile_cell(g, tl, blockIdx.x, x, y, z, x0, y0);
    if (act < 0) return;  // uniform over the workgroup
    int any = 0;
    if (act) {
        Nbr<D> nb;
        nb.init(g, x, y, z);
        unroll<0, Lat<D>::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            any |= mask[nb.at(Lat<D>::c[i][0], Lat<D>::c[i][1], Lat<D>::c[i][2])];
        });
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) tsolid[blockIdx.x] = any ? 1 : 0;
}

// tflat[w] = 1 when some cell of tile w has a porosity neighbourhood (the 3 x 3 (x 3) cells
// around it, through the periodic wrap) that is not uniform, i.e. when differenced porosity
// derivatives can be nonzero there; 0 lets the velocity correction skip the whole tile.
template <int D, typename T>
__global__ __launch_bounds__(256) void k_tile_flat(const T *__restrict__ eps, Grid g, Tiling tl,
                                                   uint8_t *__restrict__ tflat) {
    int x, y, z, x0, y0;
    const int act = tile_cell(g, tl, blockIdx.x, x, y, z, x0, y0);
    if (act < 0) return;  // uniform over the workgroup
    int bumpy = 0;
    if (act) {
        Nbr<D> nb;
        nb.init(g, x, y, z);
        const T e0 = ld(eps, nb.self());
        unroll<0, Lat<D>::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            bumpy |= ld(eps, nb.at(Lat<D>::c[i][0], Lat<D>::c[i][1], Lat<D>::c[i][2])) != e0;
        });
    }
    bumpy = __syncthreads_or(bumpy);
    if (threadIdx.x == 0) tflat[blockIdx.x] = bumpy ? 1 : 0;
}

// Initial populations, eq. (eq_bc_f_bar) with lambda = dt = 1, from the moment fields (rho, v):
// f-bar_i = (1 + 1/2) f^eq_i - (1/2) f^*_i, written in natural layout.  A 16-bit slot is
// encoded with the shift of its source cell, as a phase-0 read decodes it.
template <int D, typename T, typename P, bool SOLIDS, bool AD>
__global__ __launch_bounds__(256) void k_init(P *__restrict__ f,
                                              const P4<T> *__restrict__ m2,
                                              const T *__restrict__ eps,
                                              const T *__restrict__ muD,
                                              const T *__restrict__ muF,
                                              const uint8_t *__restrict__ mask, Grid g,
                                              Tiling tl, Phys<T> ph) {
    LBM_CELL_PROLOGUE(D)
    using L = Lat<D>;
    if constexpr (SOLIDS) {
        if (mask[n]) {
            unroll<0, L::Q>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                *at(plane(f, i, g.N), n) = P(0);
            });
            return;
        }
    }
    const Rec<T> own = load_rec<D>(m2, n, ev.at(0, 0, 0));
    const CellStatic<D, T> cs = cell_static<D, AD>(ev, ph, n, own.e);
    ProductForm<D, T> peq, pst;
    cell_equilibria<D, T, SOLIDS>(m2, ev, eps, muD, muF, mask, g, ph, nb, own, cs, peq, pst);
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const T v = T(1.5) * peq.template at<i>() - T(0.5) * pst.template at<i>();
        *at(plane(f, i, g.N), n) = encode<D, i, P>(v, load_sigma<D, SOLIDS, i, P>(mask, ev, ph, nb));
    });
}

// Create-time coefficients from FP64 host inputs staged on the device:
// mu_D = eps nu_f / kappa (mu_D_Ergun_perm), mu_F = eps C_F (mu_F_Ergun_perm).
template <typename T>
__global__ __launch_bounds__(256) void k_static(const double *__restrict__ eps_in,
                                                const double *__restrict__ kappa_in,
                                                const double *__restrict__ cf_in,
                                                T *__restrict__ eps, T *__restrict__ muD,
                                                T *__restrict__ muF, int64_t N, double nu_f) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const double e = eps_in[n];
    eps[n] = (T)e;
    muD[n] = (T)(e * nu_f / kappa_in[n]);
    muF[n] = (T)(e * cf_in[n]);
}

// Initial moment records: rho = rho_init or rho0, v = v_init or 0 (0 on solid cells); m1, when
// given, receives the same records (the lagged scheme's previous-step history at creation).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_fill_init(const double *__restrict__ rho_in,
                                                   const double *__restrict__ v_in,
                                                   const uint8_t *__restrict__ mask,
                                                   P4<T> *__restrict__ m2, P4<T> *__restrict__ m1,
                                                   int64_t N, double rho0) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const bool solid = mask && mask[n];
    T w[3] = {T(0), T(0), T(0)};
    if (!solid && v_in)
#pragma unroll
        for (int a = 0; a < D; ++a) w[a] = (T)v_in[(int64_t)a * N + n];
    const P4<T> q = pack(solid ? T(0) : (T)(rho_in ? rho_in[n] : rho0), w[0], w[1], w[2]);
    m2[n] = q;
    if (m1) m1[n] = q;
}

// Natural-layout copy of the current populations (0 on solid cells).
template <int D, typename T, typename P, bool SOLIDS, int PH, typename O>
__global__ __launch_bounds__(256) void k_export(const P *__restrict__ f,
                                                const uint8_t *__restrict__ mask,
                                                const T *__restrict__ eps, O *__restrict__ out,
                                                Grid g, Tiling tl, Phys<T> ph) {
    LBM_CELL_PROLOGUE(D)
    using L = Lat<D>;
    const bool solid = SOLIDS && mask[n];
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        if (solid) {
            out[(int64_t)i * g.N + n] = O(0);
        } else {
            const P raw = load_raw<D, SOLIDS, PH, i>(f, mask, g, nb);
            out[(int64_t)i * g.N + n] =
                decode<D, i, O>(raw, load_sigma<D, SOLIDS, i, P>(mask, ev, ph, nb));
        }
    });
}

// Populations from a natural-layout array [Q][N] (the state then reads as phase 0).
template <int D, typename T, typename P, bool SOLIDS, typename I>
__global__ __launch_bounds__(256) void k_import(P *__restrict__ f, const I *__restrict__ in,
                                                const uint8_t *__restrict__ mask,
                                                const T *__restrict__ eps, Grid g, Tiling tl,
                                                Phys<T> ph) {
    LBM_CELL_PROLOGUE(D)
    using L = Lat<D>;
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const float sig = load_sigma<D, SOLIDS, i, P>(mask, ev, ph, nb);
        if constexpr (PopFmt<P>::shifted) {
            *at(plane(f, i, g.N), n) = encode<D, i, P>(in[(int64_t)i * g.N + n], sig);
        } else {
            *at(plane(f, i, g.N), n) = (P)in[(int64_t)i * g.N + n];
        }
    });
}

// Caller-facing moments: rho and v (kind 0) or u = v / eps (kind 1), from the packed records.
template <int D, typename T, typename O>
__global__ __launch_bounds__(256) void k_moments_out(const P4<T> *__restrict__ m2,
                                                     const T *__restrict__ eps,
                                                     O *__restrict__ rho_out, O *__restrict__ v_out,
                                                     int64_t N, int kind) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const P4<T> q = m2[n];
    if (rho_out) rho_out[n] = (O)q.x;
    if (v_out) {
        const T e = eps[n];
        const T w[3] = {q.y, q.z, q.w};
#pragma unroll
        for (int a = 0; a < D; ++a) v_out[(int64_t)a * N + n] = (O)(kind ? w[a] / e : w[a]);
    }
}

// ------------------------------------------------------------------------------------------
// FP64 statistics: per-block partial sums with wavefront shuffles, then one block that adds
// the partials in a fixed order.  Slots: 0 mass, 1-3 momentum, 4 max|v|, 5 sum|v-v_prev|^2,
// 6 sum|v_prev|^2, 7 non-finite count.
// ------------------------------------------------------------------------------------------
constexpr int kStatsBlocks = 1024;
constexpr int kStatsSlots = 8;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

template <int D, typename T, typename P, bool SOLIDS, int PH>
__global__ __launch_bounds__(256) void k_stats(const P *__restrict__ f,
                                               const P4<T> *__restrict__ m2,
                                               T *__restrict__ vsnap,
                                               const uint8_t *__restrict__ mask,
                                               const T *__restrict__ eps,
                                               double *__restrict__ partial, Grid g,
                                               Phys<T> ph) {
    using L = Lat<D>;
    double acc[kStatsSlots] = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint32_t stride = gridDim.x * 256u;
    for (uint32_t n = blockIdx.x * 256u + threadIdx.x; n < g.N; n += stride) {
        if (SOLIDS && mask[n]) continue;
        const int x = (int)(n % (uint32_t)g.nx);
        const int y = (int)((n / (uint32_t)g.nx) % (uint32_t)g.ny);
        const int z = (int)(n / ((uint32_t)g.nx * (uint32_t)g.ny));
        Nbr<D> nb;
        nb.init(g, x, y, z);
        const EpsGlobal<D, T> ev{eps, &nb};
        // every population decoded to FP64 (exact for each storage form) and summed in FP64
        double cm = 0.0;
        unroll<0, L::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const P raw = load_raw<D, SOLIDS, PH, i>(f, mask, g, nb);
            cm = cm + decode<D, i, double>(raw, load_sigma<D, SOLIDS, i, P>(mask, ev, ph, nb));
        });
        acc[0] += cm;
        double vv = 0.0;
        const P4<T> q = m2[n];
        const double r = (double)q.x;
        const T w[3] = {q.y, q.z, q.w};
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double va = (double)w[a];
            const double sa = (double)vsnap[(size_t)a * g.N + n];
            acc[1 + a] += r * va;
            vv += va * va;
            acc[5] += (va - sa) * (va - sa);
            acc[6] += sa * sa;
            vsnap[(size_t)a * g.N + n] = w[a];
        }
        // a cell counts once, whether its populations, its velocity or both are not finite
        if (!isfinite(cm) || !isfinite(vv)) acc[7] += 1.0;
        if (isfinite(vv)) acc[4] = fmax(acc[4], sqrt(vv));
    }
    __shared__ double red[4][kStatsSlots];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kStatsSlots; ++k) {
        const double s = k == 4 ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kStatsSlots) {
        const int k = threadIdx.x;
        double s = red[0][k];
        for (int w = 1; w < 4; ++w) s = k == 4 ? fmax(s, red[w][k]) : s + red[w][k];
        partial[(int64_t)blockIdx.x * kStatsSlots + k] = s;
    }
}

static __global__ __launch_bounds__(256) void k_stats_final(const double *__restrict__ partial,
                                                     int nblocks, double *__restrict__ out) {
    double acc[kStatsSlots] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int k = 0; k < kStatsSlots; ++k) {
            const double p = partial[(int64_t)b * kStatsSlots + k];
            acc[k] = k == 4 ? fmax(acc[k], p) : acc[k] + p;
        }
    }
    __shared__ double red[4][kStatsSlots];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kStatsSlots; ++k) {
        const double s = k == 4 ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kStatsSlots) {
        const int k = threadIdx.x;
        double s = red[0][k];
        for (int w = 1; w < 4; ++w) s = k == 4 ? fmax(s, red[w][k]) : s + red[w][k];
        out[k] = s;
    }
}

}  // namespace lbm
