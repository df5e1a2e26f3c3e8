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
// Floating-point: the library is built with -ffp-contract=off and every expression below is
// written in the evaluation order of the CPU reference, so FP64 results agree bit for bit.
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
    int64_t N;
};

template <typename T>
struct Phys {
    T RT;          // lattice temperature
    T omr;         // 1 - 3 RT
    T nu_ref;      // nu_eff(eps) = nu_ref * eps^nu_pow
    T eta;         // effective bulk viscosity (Phi^eta)
    T two_over_D;  // 2 / D
    T b[3];        // body acceleration
    int nu_pow;    // -1, 0, 1
    int eta_on;    // Phi^eta switched on
};

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

__device__ __forceinline__ int64_t cell_index(const Grid &g, int x, int y, int z) {
    return (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
}

// Neighbour of (x,y,z) displaced by k (|k| <= 2) along axis a.
__device__ __forceinline__ int64_t axis_neighbor(const Grid &g, int x, int y, int z, int a, int k) {
    if (k == 1 || k == -1) {
        if (a == 0) x = wrap1(x, k, g.nx);
        else if (a == 1) y = wrap1(y, k, g.ny);
        else z = wrap1(z, k, g.nz);
    } else {
        if (a == 0) x = wrapk(x, k, g.nx);
        else if (a == 1) y = wrapk(y, k, g.ny);
        else z = wrapk(z, k, g.nz);
    }
    return cell_index(g, x, y, z);
}

// ------------------------------------------------------------------------------------------
// AA-pattern population access
// ------------------------------------------------------------------------------------------
template <int D, bool SOLIDS, int PH, int I, typename T>
__device__ __forceinline__ T load_pop(const T *__restrict__ f, const uint8_t *__restrict__ mask,
                                      const Grid &g, int x, int y, int z, int64_t n) {
    using L = Lat<D>;
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    if constexpr (PH == 0 || (cx == 0 && cy == 0 && cz == 0)) {
        return f[(int64_t)I * g.N + n];
    } else {
        const int sx = wrap1(x, -cx, g.nx), sy = wrap1(y, -cy, g.ny);
        const int sz = D == 3 ? wrap1(z, -cz, g.nz) : z;
        const int64_t s = cell_index(g, sx, sy, sz);
        if constexpr (SOLIDS) {
            if (mask[s]) return f[(int64_t)I * g.N + n];
        }
        return f[(int64_t)L::opp[I] * g.N + s];
    }
}

template <int D, bool SOLIDS, int PH, int I, typename T>
__device__ __forceinline__ void store_pop(T *__restrict__ f, const uint8_t *__restrict__ mask,
                                          const Grid &g, int x, int y, int z, int64_t n, T val) {
    using L = Lat<D>;
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    if constexpr (PH == 0 || (cx == 0 && cy == 0 && cz == 0)) {
        f[(int64_t)L::opp[I] * g.N + n] = val;
    } else {
        const int dx = wrap1(x, cx, g.nx), dy = wrap1(y, cy, g.ny);
        const int dz = D == 3 ? wrap1(z, cz, g.nz) : z;
        const int64_t d = cell_index(g, dx, dy, dz);
        if constexpr (SOLIDS) {
            if (mask[d]) {
                f[(int64_t)L::opp[I] * g.N + n] = val;
                return;
            }
        }
        f[(int64_t)I * g.N + d] = val;
    }
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
        r.nu = ph.nu_ref / e;
        r.dnu = -ph.nu_ref / (e * e);
    } else if (ph.nu_pow == 1) {
        r.nu = ph.nu_ref * e;
        r.dnu = ph.nu_ref;
    } else {
        r.nu = ph.nu_ref;
        r.dnu = T(0);
    }
    r.beta = T(1) / (T(1) + (T(2) * r.nu) / ph.RT);
    return r;
}

// Porosity gradient and Hessian by central differences (eps is defined on every cell).
template <int D, typename T>
__device__ __forceinline__ void porosity_derivatives(const T *__restrict__ eps, const Grid &g,
                                                     int x, int y, int z, T e0, T ge[3],
                                                     T H[3][3]) {
    unroll<0, D>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        const T ep = eps[axis_neighbor(g, x, y, z, a, 1)];
        const T em = eps[axis_neighbor(g, x, y, z, a, -1)];
        ge[a] = (ep - em) * T(0.5);
        H[a][a] = (ep - T(2) * e0) + em;
    });
    unroll<0, D>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        unroll<a + 1, D>([&](auto ib) {
            constexpr int b = decltype(ib)::value;
            int c[3];
            auto at = [&](int ka, int kb) {
                c[0] = x; c[1] = y; c[2] = z;
                const int na = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
                const int nb = b == 0 ? g.nx : (b == 1 ? g.ny : g.nz);
                c[a] = wrap1(c[a], ka, na);
                c[b] = wrap1(c[b], kb, nb);
                return eps[cell_index(g, c[0], c[1], c[2])];
            };
            const T pp = at(1, 1), pm = at(1, -1), mp = at(-1, 1), mm = at(-1, -1);
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

// Moment record of one cell: intrinsic density, porosity, velocity.
template <typename T>
struct Rec {
    T r, e, w[3];
};

template <int D, typename T>
__device__ __forceinline__ Rec<T> load_rec(const T *__restrict__ rho, const T *__restrict__ w,
                                           const T *__restrict__ eps, const Grid &g, int64_t m) {
    Rec<T> q;
    q.r = rho[m];
    q.e = eps[m];
#pragma unroll
    for (int b = 0; b < D; ++b) q.w[b] = w[(int64_t)b * g.N + m];
    return q;
}

// Variable-porosity viscous correction Delta_nu(m) at the cell, m = rho w / eps built from the
// record fields, eq. (porosity_correction_expanded):
//   nu {[H + tr(H) I] m + (div m) grad eps + (grad m) grad eps}
//     + nu' [|grad eps|^2 m + (m . grad eps) grad eps],   [(grad m) grad eps]_a = sum_b d_b m_a d_b eps.
// own: the cell's record; nb[a][0|1]: records of the -/+ neighbours along axis a.
template <int D, typename T, bool SOLIDS>
__device__ __forceinline__ void delta_nu(const T *__restrict__ rho, const T *__restrict__ w,
                                         const T *__restrict__ eps,
                                         const uint8_t *__restrict__ mask, const Grid &g, int x,
                                         int y, int z, const Rec<T> &own, const Rec<T> nb[3][2],
                                         const bool fl[3][2], const T ge[3], const T H[3][3],
                                         const Visc<T> &vs, T out[3]) {
    T mo[3];
#pragma unroll
    for (int b = 0; b < D; ++b) mo[b] = (own.r * own.w[b]) / own.e;
    T J[3][3];  // J[b][a] = d_a m_b
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T mm[3], mp[3];
#pragma unroll
        for (int b = 0; b < D; ++b) {
            mm[b] = (nb[a][0].r * nb[a][0].w[b]) / nb[a][0].e;
            mp[b] = (nb[a][1].r * nb[a][1].w[b]) / nb[a][1].e;
        }
        if (!SOLIDS || (fl[a][0] && fl[a][1])) {
#pragma unroll
            for (int b = 0; b < D; ++b) J[b][a] = (mp[b] - mm[b]) * T(0.5);
        } else {
            bool f5[5] = {false, fl[a][0], true, fl[a][1], false};
            Rec<T> r2[2];
            if (fl[a][1] && !fl[a][0]) {
                const int64_t p2 = axis_neighbor(g, x, y, z, a, 2);
                f5[4] = !mask[p2];
                if (f5[4]) r2[1] = load_rec<D>(rho, w, eps, g, p2);
            }
            if (fl[a][0] && !fl[a][1]) {
                const int64_t m2 = axis_neighbor(g, x, y, z, a, -2);
                f5[0] = !mask[m2];
                if (f5[0]) r2[0] = load_rec<D>(rho, w, eps, g, m2);
            }
#pragma unroll
            for (int b = 0; b < D; ++b) {
                T v5[5];
                v5[0] = f5[0] ? (r2[0].r * r2[0].w[b]) / r2[0].e : T(0);
                v5[1] = mm[b];
                v5[2] = mo[b];
                v5[3] = mp[b];
                v5[4] = f5[4] ? (r2[1].r * r2[1].w[b]) / r2[1].e : T(0);
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

// Load the own record and the 2D axis neighbours with their fluid flags.
template <int D, typename T, bool SOLIDS>
__device__ __forceinline__ void load_stencil(const T *__restrict__ rho, const T *__restrict__ w,
                                             const T *__restrict__ eps,
                                             const uint8_t *__restrict__ mask, const Grid &g,
                                             int x, int y, int z, Rec<T> nb[3][2],
                                             bool fl[3][2]) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int64_t m = axis_neighbor(g, x, y, z, a, s ? 1 : -1);
            nb[a][s] = load_rec<D>(rho, w, eps, g, m);
            fl[a][s] = SOLIDS ? !mask[m] : true;
        }
    }
}

// Derivative along axis a of a scalar built from a record (Phi^ext's flux, or v_a).
template <int D, typename T, bool SOLIDS, typename F>
__device__ __forceinline__ T record_deriv(const T *__restrict__ rho, const T *__restrict__ w,
                                          const T *__restrict__ eps,
                                          const uint8_t *__restrict__ mask, const Grid &g, int x,
                                          int y, int z, int a, const Rec<T> &own,
                                          const Rec<T> nb[3][2], const bool fl[3][2], F fn) {
    const T vm = fn(nb[a][0]), vp = fn(nb[a][1]);
    if (!SOLIDS || (fl[a][0] && fl[a][1])) return (vp - vm) * T(0.5);
    bool f5[5] = {false, fl[a][0], true, fl[a][1], false};
    T v5[5] = {T(0), vm, fn(own), vp, T(0)};
    if (fl[a][1] && !fl[a][0]) {
        const int64_t p2 = axis_neighbor(g, x, y, z, a, 2);
        f5[4] = !mask[p2];
        if (f5[4]) v5[4] = fn(load_rec<D>(rho, w, eps, g, p2));
    }
    if (fl[a][0] && !fl[a][1]) {
        const int64_t m2 = axis_neighbor(g, x, y, z, a, -2);
        f5[0] = !mask[m2];
        if (f5[0]) v5[0] = fn(load_rec<D>(rho, w, eps, g, m2));
    }
    return deriv_rule(v5, f5);
}

// Equilibrium and shifted-equilibrium arguments of one cell from the moment fields (rho, v):
// acceleration (accel), Phi^ext (ex_corr), Phi^eta (eta_corr), then xi, P (xi_alpha_eq,
// P_alpha_alpha_eq) and xi*, P* (xi_alpha_*, P_aa_*) with lambda = 1.
template <int D, typename T, bool SOLIDS>
__device__ __forceinline__ void forcing_args(const T *__restrict__ rho, const T *__restrict__ v,
                                             const T *__restrict__ eps,
                                             const T *__restrict__ muD,
                                             const T *__restrict__ muF,
                                             const uint8_t *__restrict__ mask, const Grid &g,
                                             const Phys<T> &ph, int x, int y, int z, int64_t n,
                                             Rec<T> &own, Visc<T> &vs, T xi[3], T P[3], T xs[3],
                                             T Ps[3]) {
    own = load_rec<D>(rho, v, eps, g, n);
    Rec<T> nb[3][2];
    bool fl[3][2];
    load_stencil<D, T, SOLIDS>(rho, v, eps, mask, g, x, y, z, nb, fl);
    T ge[3], H[3][3];
    porosity_derivatives<D>(eps, g, x, y, z, own.e, ge, H);
    vs = viscosity(ph, own.e);
    T dm[3] = {T(0), T(0), T(0)};
    delta_nu<D, T, SOLIDS>(rho, v, eps, mask, g, x, y, z, own, nb, fl, ge, H, vs, dm);
    T s = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) s = s + own.w[a] * own.w[a];
    const T vm = sqrt(s);
    const T md = muD[n], mf = muF[n];
    T acc[3];
#pragma unroll
    for (int a = 0; a < D; ++a)
        acc[a] = (((own.e * ph.b[a] - md * own.w[a]) - (mf * vm) * own.w[a]) + ph.RT * ge[a]) +
                 dm[a] / own.r;
    T phx[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T omr = ph.omr;
        auto gext = [a, omr](const Rec<T> &q) {
            const T va = q.w[a];
            return (q.r * va) * omr - (q.r * ((va * va) * va)) / (q.e * q.e);
        };
        phx[a] = record_deriv<D, T, SOLIDS>(rho, v, eps, mask, g, x, y, z, a, own, nb, fl, gext);
    }
    T pheta = T(0);
    if (ph.eta_on) {
        T divv = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            auto va = [a](const Rec<T> &q) { return q.w[a]; };
            divv = divv + record_deriv<D, T, SOLIDS>(rho, v, eps, mask, g, x, y, z, a, own, nb,
                                                       fl, va);
        }
        pheta = ((own.r * ph.RT) * (ph.two_over_D - ph.eta / vs.nu)) * divv;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xi[a] = own.w[a] / own.e;
        P[a] = xi[a] * xi[a] + ph.RT;
        xs[a] = (own.w[a] + acc[a]) / own.e;
        Ps[a] = (xs[a] * xs[a] + ph.RT) + (T(1) / (own.e * own.r)) * (phx[a] + pheta);
    }
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

// ------------------------------------------------------------------------------------------
// Kernels.  Launch: block (64, 4, 1) over (x, y), grid z = cells along z.
// ------------------------------------------------------------------------------------------
#define LBM_CELL_PROLOGUE                                             \
    const int x = blockIdx.x * 64 + threadIdx.x;                     \
    const int y = blockIdx.y * 4 + threadIdx.y;                      \
    const int z = blockIdx.z;                                        \
    if (x >= g.nx || y >= g.ny) return;                              \
    const int64_t n = cell_index(g, x, y, z);

// Pass one: density (transformed_density_moment), transformed momentum
// (transformed_momentum_moment), v^(0) (v_(0)) and the closed-form drag solve v^(1)
// (v_(1), velocity_coefficients); writes rho [N] and v^(1) [D][N].
template <int D, typename T, bool SOLIDS, int PH>
__global__ __launch_bounds__(256) void k_moments(const T *__restrict__ f,
                                                 const T *__restrict__ eps,
                                                 const T *__restrict__ muD,
                                                 const T *__restrict__ muF,
                                                 const uint8_t *__restrict__ mask,
                                                 T *__restrict__ rho_out, T *__restrict__ v1_out,
                                                 Grid g, Phys<T> ph) {
    LBM_CELL_PROLOGUE
    using L = Lat<D>;
    if constexpr (SOLIDS) {
        if (mask[n]) {
            rho_out[n] = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) v1_out[(int64_t)a * g.N + n] = T(0);
            return;
        }
    }
    T fi[L::Q];
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        fi[i] = load_pop<D, SOLIDS, PH, i>(f, mask, g, x, y, z, n);
    });
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
    const T e = eps[n];
    const T rho = S / e;
    T v0[3];
    unroll<0, D>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        const T ge = (eps[axis_neighbor(g, x, y, z, a, 1)] - eps[axis_neighbor(g, x, y, z, a, -1)]) *
                     T(0.5);
        v0[a] = Pi[a] / rho + T(0.5) * (e * ph.b[a] + ph.RT * ge);
    });
    const T c1 = T(1) + T(0.5) * muD[n];
    const T c2 = T(0.5) * muF[n];
    T s = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) s = s + v0[a] * v0[a];
    const T vm = sqrt(s);
    const T den = c1 + sqrt(c1 * c1 + (T(4) * c2) * vm);
    rho_out[n] = rho;
#pragma unroll
    for (int a = 0; a < D; ++a) v1_out[(int64_t)a * g.N + n] = (T(2) * v0[a]) / den;
}

// Velocity correction (v_final): v = v^(1) + Delta_nu(rho v^(1) / eps) / (2 rho).
template <int D, typename T, bool SOLIDS>
__global__ __launch_bounds__(256) void k_vcorrect(const T *__restrict__ rho,
                                                  const T *__restrict__ v1,
                                                  const T *__restrict__ eps,
                                                  const uint8_t *__restrict__ mask,
                                                  T *__restrict__ v_out, Grid g, Phys<T> ph) {
    LBM_CELL_PROLOGUE
    if constexpr (SOLIDS) {
        if (mask[n]) {
#pragma unroll
            for (int a = 0; a < D; ++a) v_out[(int64_t)a * g.N + n] = T(0);
            return;
        }
    }
    const Rec<T> own = load_rec<D>(rho, v1, eps, g, n);
    Rec<T> nb[3][2];
    bool fl[3][2];
    load_stencil<D, T, SOLIDS>(rho, v1, eps, mask, g, x, y, z, nb, fl);
    T ge[3], H[3][3];
    porosity_derivatives<D>(eps, g, x, y, z, own.e, ge, H);
    const Visc<T> vs = viscosity(ph, own.e);
    T dn[3];
    delta_nu<D, T, SOLIDS>(rho, v1, eps, mask, g, x, y, z, own, nb, fl, ge, H, vs, dn);
#pragma unroll
    for (int a = 0; a < D; ++a)
        v_out[(int64_t)a * g.N + n] = own.w[a] + dn[a] / (T(2) * own.r);
}

// Forcing, collision (dicrete_scheme, momentum_rate with lambda = dt = 1) and streaming with
// halfway bounce-back, in place:
//   f^pc_i = f_i + 2 beta (f^eq_i - f_i) + (1 - beta)(f^*_i - f^eq_i).
template <int D, typename T, bool SOLIDS, int PH>
__global__ __launch_bounds__(256) void k_collide(T *__restrict__ f, const T *__restrict__ rho,
                                                 const T *__restrict__ v,
                                                 const T *__restrict__ eps,
                                                 const T *__restrict__ muD,
                                                 const T *__restrict__ muF,
                                                 const uint8_t *__restrict__ mask, Grid g,
                                                 Phys<T> ph) {
    LBM_CELL_PROLOGUE
    using L = Lat<D>;
    if constexpr (SOLIDS) {
        if (mask[n]) return;
    }
    T fi[L::Q];
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        fi[i] = load_pop<D, SOLIDS, PH, i>(f, mask, g, x, y, z, n);
    });
    Rec<T> own;
    Visc<T> vs;
    T xi[3], P[3], xs[3], Ps[3];
    forcing_args<D, T, SOLIDS>(rho, v, eps, muD, muF, mask, g, ph, x, y, z, n, own, vs, xi, P,
                               xs, Ps);
    const T er = own.e * own.r;
    ProductForm<D, T> peq, pst;
    peq.init(er, xi, P);
    pst.init(er, xs, Ps);
    const T two_beta = T(2) * vs.beta;
    const T omb = T(1) - vs.beta;
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const T feq = peq.template at<i>();
        const T fst = pst.template at<i>();
        const T fpc = (fi[i] + two_beta * (feq - fi[i])) + omb * (fst - feq);
        store_pop<D, SOLIDS, PH, i>(f, mask, g, x, y, z, n, fpc);
    });
}

// Initial populations, eq. (eq_bc_f_bar) with lambda = dt = 1, from the moment fields (rho, v):
// f-bar_i = (1 + 1/2) f^eq_i - (1/2) f^*_i, written in natural layout.
template <int D, typename T, bool SOLIDS>
__global__ __launch_bounds__(256) void k_init(T *__restrict__ f, const T *__restrict__ rho,
                                              const T *__restrict__ v,
                                              const T *__restrict__ eps,
                                              const T *__restrict__ muD,
                                              const T *__restrict__ muF,
                                              const uint8_t *__restrict__ mask, Grid g,
                                              Phys<T> ph) {
    LBM_CELL_PROLOGUE
    using L = Lat<D>;
    if constexpr (SOLIDS) {
        if (mask[n]) {
            unroll<0, L::Q>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                f[(int64_t)i * g.N + n] = T(0);
            });
            return;
        }
    }
    Rec<T> own;
    Visc<T> vs;
    T xi[3], P[3], xs[3], Ps[3];
    forcing_args<D, T, SOLIDS>(rho, v, eps, muD, muF, mask, g, ph, x, y, z, n, own, vs, xi, P,
                               xs, Ps);
    const T er = own.e * own.r;
    ProductForm<D, T> peq, pst;
    peq.init(er, xi, P);
    pst.init(er, xs, Ps);
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        f[(int64_t)i * g.N + n] = T(1.5) * peq.template at<i>() - T(0.5) * pst.template at<i>();
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

// Initial moment fields: rho = rho_init or rho0, v = v_init or 0 (0 on solid cells).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_fill_init(const double *__restrict__ rho_in,
                                                   const double *__restrict__ v_in,
                                                   const uint8_t *__restrict__ mask,
                                                   T *__restrict__ rho, T *__restrict__ v,
                                                   int64_t N, double rho0) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const bool solid = mask && mask[n];
    rho[n] = solid ? T(0) : (T)(rho_in ? rho_in[n] : rho0);
#pragma unroll
    for (int a = 0; a < D; ++a) v[(int64_t)a * N + n] = solid ? T(0) : (T)(v_in ? v_in[(int64_t)a * N + n] : 0.0);
}

// Natural-layout copy of the current populations (0 on solid cells).
template <int D, typename T, bool SOLIDS, int PH, typename O>
__global__ __launch_bounds__(256) void k_export(const T *__restrict__ f,
                                                const uint8_t *__restrict__ mask,
                                                O *__restrict__ out, Grid g) {
    LBM_CELL_PROLOGUE
    using L = Lat<D>;
    const bool solid = SOLIDS && mask[n];
    unroll<0, L::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        out[(int64_t)i * g.N + n] = solid ? O(0) : (O)load_pop<D, SOLIDS, PH, i>(f, mask, g, x, y, z, n);
    });
}

template <typename T, typename I>
__global__ __launch_bounds__(256) void k_import(T *__restrict__ f, const I *__restrict__ in,
                                                int64_t total) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < total) f[k] = (T)in[k];
}

// Caller-facing moments: rho and v (kind 0) or u = v / eps (kind 1).
template <int D, typename T, typename O>
__global__ __launch_bounds__(256) void k_moments_out(const T *__restrict__ rho,
                                                     const T *__restrict__ v,
                                                     const T *__restrict__ eps,
                                                     O *__restrict__ rho_out, O *__restrict__ v_out,
                                                     int64_t N, int kind) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    if (rho_out) rho_out[n] = (O)rho[n];
    if (v_out) {
        const T e = eps[n];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const T va = v[(int64_t)a * N + n];
            v_out[(int64_t)a * N + n] = (O)(kind ? va / e : va);
        }
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

template <int D, typename T, bool SOLIDS, int PH>
__global__ __launch_bounds__(256) void k_stats(const T *__restrict__ f, const T *__restrict__ rho,
                                               const T *__restrict__ v, T *__restrict__ vsnap,
                                               const uint8_t *__restrict__ mask,
                                               double *__restrict__ partial, Grid g) {
    using L = Lat<D>;
    double acc[kStatsSlots] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < g.N; n += stride) {
        if (SOLIDS && mask[n]) continue;
        const int x = (int)(n % g.nx);
        const int y = (int)((n / g.nx) % g.ny);
        const int z = (int)(n / ((int64_t)g.nx * g.ny));
        T cell = T(0);
        unroll<0, L::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            cell = cell + load_pop<D, SOLIDS, PH, i>(f, mask, g, x, y, z, n);
        });
        const double cm = (double)cell;
        acc[0] += cm;
        if (!isfinite(cm)) acc[7] += 1.0;
        double vv = 0.0;
        const double r = (double)rho[n];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double va = (double)v[(int64_t)a * g.N + n];
            const double sa = (double)vsnap[(int64_t)a * g.N + n];
            acc[1 + a] += r * va;
            vv += va * va;
            acc[5] += (va - sa) * (va - sa);
            acc[6] += sa * sa;
            vsnap[(int64_t)a * g.N + n] = v[(int64_t)a * g.N + n];
        }
        if (!isfinite(vv)) acc[7] += 1.0;
        else acc[4] = fmax(acc[4], sqrt(vv));
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

__global__ __launch_bounds__(256) void k_stats_final(const double *__restrict__ partial,
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
