// lbm_host.hpp -- host-side internals shared by the solver and the request server: error
// reporting, the workspace layout, the solver handle and the tile geometry.
#pragma once

#include "lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <type_traits>

#include "lbm_device.hpp"

namespace lbmh {

inline thread_local std::string g_err;

inline int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(LBM_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

#define LAUNCH_CHECK()                                                                  \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess)                                                           \
            return fail(LBM_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t f, eps, muD, muF, mask, m1[2], m2[2], vsnap, part, res;
    size_t bcell, bcode, bval;  // boundary-node list (wet-node boundaries)
    size_t m0, mx;              // (rho, v_0) records and a second velocity buffer (Picard)
    size_t deps;                // analytic porosity derivatives, D + D(D+1)/2 planes
    size_t tsolid;              // per-tile flag: a solid cell within one cell of the tile
    size_t tflat;               // per-tile flag: a porosity gradient somewhere in the tile
    size_t total;
};

// sp: bytes per population value; s: bytes per value of the static fields and moment records.
// ntiles: workgroups of the tiled passes (solid runs keep one flag byte per tile).
inline Layout make_layout(int Q, int D, size_t N, size_t sp, size_t s, bool solids, bool lagged,
                          size_t ntiles, size_t nbnodes = 0, bool picard = false,
                          bool analytic = false) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    // the population region also stages the FP64 inputs at creation (up to 4 arrays of N)
    L.f = take(std::max((size_t)Q * N * sp, 4 * N * sizeof(double)));
    L.eps = take(N * s);
    L.muD = take(N * s);
    L.muF = take(N * s);
    L.mask = solids ? take(N) : 0;
    // packed (rho, v^(1)) and (rho, v) records; the lagged scheme keeps a second pair so that
    // one step reads the previous records while it writes the new ones
    L.m1[0] = take(4 * N * s);
    L.m2[0] = take(4 * N * s);
    L.m1[1] = lagged ? take(4 * N * s) : L.m1[0];
    L.m2[1] = lagged ? take(4 * N * s) : L.m2[0];
    L.vsnap = take((size_t)D * N * s);
    L.part = take((size_t)lbm::kStatsBlocks * lbm::kStatsSlots * sizeof(double));
    L.res = take(lbm::kStatsSlots * sizeof(double));
    L.bcell = nbnodes ? take(nbnodes * sizeof(uint32_t)) : 0;
    L.bcode = nbnodes ? take(nbnodes * sizeof(uint32_t)) : 0;
    L.bval = nbnodes ? take(nbnodes * 4 * s) : 0;
    L.m0 = picard ? take(4 * N * s) : 0;
    L.mx = picard ? take(4 * N * s) : 0;
    L.deps = analytic ? take((size_t)(D + D * (D + 1) / 2) * N * s) : 0;
    L.tsolid = solids ? take(ntiles) : 0;
    L.tflat = analytic ? 0 : take(ntiles);
    L.total = off;
    return L;
}

inline bool is_finite(double x) { return std::isfinite(x); }

}  // namespace lbmh

struct lbm_solver {
    int lattice, D, Q, storage;
    int nx, ny, nz;
    int64_t N;
    bool solids;
    hipStream_t stream;
    char *ws;
    lbmh::Layout L;
    int64_t step;
    int phase;  // AA-pattern layout: 0 natural, 1 swapped
    int scheme;
    int cur;        // record pair that holds the previous step's moments (lagged scheme)
    bool have_prev; // whether that pair is valid (lagged scheme)
    double RT, nu_f, nu_eff_ref, eta_eff, b[3], rho0;
    int nu_eff_pow;
    int shift;          // 16-bit population shift (LBM_SHIFT_*)
    uint32_t nb;        // boundary nodes
    bool bc_outflow, bc_vp;  // outflow nodes, velocity or pressure nodes present
    bool bc_visc;            // face velocity nodes whose density takes the viscous term
    int bc_scheme, bc_rho_rule;
    int picard_iters;
    double picard_omega;
    bool analytic;      // analytic porosity derivatives in L.deps
    lbm::Tiling tiles;  // 256-cell tiles, blocked, in XCD-contiguous ranges
    bool fused_vc;      // velocity correction inside the collision pass (k_collide_vc)
    bool solid_occ;     // runs with solids: under a quarter of the tiles solid-aware
    lbm::ZTiling ztiles;
    int device;         // HIP device current at creation
};

namespace lbmh {

// Lattice temperature in the arithmetic type.  In FP32 it is rounded so that 1 - RT is exact
// (RT' = 1 - fl(1 - fl(RT)), exact by Sterbenz's lemma): then the three factors 1 - P and
// (P -/+ xi)/2 of each axis of the product-form equilibrium sum to exactly 1 for a cell at rest.
// With the nearest float of 1/3 they sum to 1 - 3e-8 per axis, which drains about 1e-7 of the
// mass per step.  The change of RT is below 2 ulp (1.2e-7 relative for 1/3); FP64 keeps RT.
template <typename T>
T lattice_temperature(double RT) {
    if constexpr (std::is_same_v<T, float>) {
        const float rt = (float)RT;
        const float c = 1.0f - rt;  // rounded: 1 - rt needs one bit more than a float for 1/3
        return 1.0f - c;            // exact (Sterbenz), and 1 - (1 - c) == c
    } else {
        return (T)RT;
    }
}

template <typename T>
lbm::Phys<T> phys_of(const lbm_solver *h) {
    lbm::Phys<T> ph;
    ph.RT = lattice_temperature<T>(h->RT);
    ph.omr = (T)(1.0 - 3.0 * h->RT);
    ph.nu_ref = (T)h->nu_eff_ref;
    ph.eta_on = std::isnan(h->eta_eff) ? 0 : 1;
    ph.eta = ph.eta_on ? (T)h->eta_eff : T(0);
    ph.two_over_D = (T)(2.0 / (double)h->D);
    for (int a = 0; a < 3; ++a) ph.b[a] = (T)h->b[a];
    ph.nu_pow = h->nu_eff_pow;
    ph.rho0 = (T)h->rho0;
    ph.shift_porous = h->shift == LBM_SHIFT_POROUS ? 1 : 0;
    ph.deps = h->analytic ? reinterpret_cast<const T *>(h->ws + h->L.deps) : nullptr;
    ph.dN = (uint32_t)h->N;
    return ph;
}

inline lbm::Grid grid_of(const lbm_solver *h) { return lbm::Grid{h->nx, h->ny, h->nz, (uint32_t)h->N}; }


inline dim3 flat_grid(int64_t total) { return dim3((unsigned)((total + 255) / 256)); }

// Tiles of the fused correction-collision pass: tx x ty cells (nx % tx == 0, ny % ty == 0),
// marched through chunks of zc z-planes, the eight XCDs taking contiguous ranges of the
// x-fastest, then y, then chunk order (neighbouring tiles in y share their ring rows in the
// XCD's L2).  One workgroup fills a CU (LDS rings of 143 KB in FP32, 114 KB for the 16-bit
// forms, 146 KB in FP64), so the chunks are as long as 256 workgroups allow, between 8 and 128
// planes: long chunks correct and stage fewer end planes (256^3 box, FP32, an earlier version
// of the kernel: chunks of 32, 64 and 128 planes 0.924, 0.936 and 0.906 ms).
inline lbm::ZTiling make_ztiling(int nx, int ny, int nz, int tx, int ty) {
    lbm::ZTiling z{};
    z.ntx = nx / tx;
    z.nty = ny / ty;
    const int64_t cols = (int64_t)z.ntx * z.nty;
    z.zc = (int)std::min<int64_t>(nz, std::max<int64_t>(8, std::min<int64_t>(128, cols * nz / 256)));
    z.nch = (nz + z.zc - 1) / z.zc;
    z.per = (uint32_t)((cols * z.nch + 7) / 8);
    return z;
}

// Tiles of the cell passes.  Rectangular tiles (256 x 1, 128 x 2 or 64 x 4 cells) when the x
// extent is a multiple of 64 (or the caller asks for them); packed rows otherwise, so that rows
// of, say, 70 cells do not leave most of a second wave idle.
// Width of the rectangular row tiles for an x extent nx.
inline int rect_tile_x(int nx) { return nx >= 192 ? 256 : (nx >= 96 ? 128 : 64); }

inline lbm::Tiling make_tiling(int nx, int ny, int nz, bool packed_ok = false) {
    lbm::Tiling t{};
    if (packed_ok && nx % 64 != 0) {
        t.packed = 1;
        t.tx = 256;
        t.ltx = 8;
        t.ty = 1;
        t.ntx = 1;
        t.pn = (uint32_t)nx * (uint32_t)ny;
        t.nty = (int)((t.pn + 255u) / 256u);
        t.mnx = nx >= 2 ? ~uint64_t(0) / (uint64_t)nx + 1 : 0;
    } else {
        t.tx = rect_tile_x(nx);
        t.ltx = t.tx == 256 ? 8 : (t.tx == 128 ? 7 : 6);
        t.ty = 256 / t.tx;
        t.ntx = (nx + t.tx - 1) / t.tx;
        t.nty = (ny + t.ty - 1) / t.ty;
    }
    t.ntz = nz;
    const int by = 64, bz = 4;  // tile rows per block along y and z (measured best on 256^3)
    t.by = std::min(by, t.nty);
    t.bz = std::min(bz, t.ntz);
    t.nby = (t.nty + t.by - 1) / t.by;
    t.nbz = (t.ntz + t.bz - 1) / t.bz;
    const int64_t nt = (int64_t)t.ntx * t.by * t.bz * t.nby * t.nbz;
    t.per = (uint32_t)((nt + 7) / 8);
    return t;
}

inline dim3 cell_tiles(const lbm_solver *h) { return dim3((unsigned)(8 * (int64_t)h->tiles.per)); }

template <typename T>
T *ws_ptr(const lbm_solver *h, size_t off) {
    return reinterpret_cast<T *>(h->ws + off);
}

inline const uint8_t *mask_ptr(const lbm_solver *h) {
    return h->solids ? reinterpret_cast<const uint8_t *>(h->ws + h->L.mask) : nullptr;
}

inline const uint8_t *tsolid_ptr(const lbm_solver *h) {
    return h->solids ? reinterpret_cast<const uint8_t *>(h->ws + h->L.tsolid) : nullptr;
}

// Flat-tile flags exist for differenced porosity derivatives only (analytic runs: null).
inline const uint8_t *tflat_ptr(const lbm_solver *h) {
    return h->analytic ? nullptr : reinterpret_cast<const uint8_t *>(h->ws + h->L.tflat);
}

// Enqueue the statistics of the current state into res (8 doubles, the lbm_stats slots) with the
// per-block partial sums in part, without synchronising; defined with the solver kernels.
int enqueue_stats(lbm_solver *h, double *part, double *res);

// The same, with the partial sums and the result in the solver's workspace.
inline int enqueue_stats(lbm_solver *h) {
    return enqueue_stats(h, ws_ptr<double>(h, h->L.part), ws_ptr<double>(h, h->L.res));
}

}  // namespace lbmh

