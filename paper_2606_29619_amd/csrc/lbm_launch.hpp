// lbm_launch.hpp -- kernel launchers and the dispatch of the solver's passes over the run's
// configuration (lattice, arithmetic and storage types, solids, AA phase, derivative source).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbm_bc.hpp"
#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbmh {

// ---- kernel launchers, dispatched on (lattice, arithmetic type T, population storage type P,
// solids, phase, derivative source) -------------------------------------------------------------
template <int D, typename T, typename P, bool S, int PH, bool AD>
void launch_moments(const lbm_solver *h, size_t m1_out) {
    auto ph = phys_of<T>(h);
    lbm::P4<T> *m0 = h->picard_iters ? ws_ptr<lbm::P4<T>>(h, h->L.m0) : nullptr;
    hipLaunchKernelGGL((lbm::k_moments<D, T, P, S, PH, AD>), cell_tiles(h), dim3(256), 0, h->stream,
                       ws_ptr<const P>(h, h->L.f), ws_ptr<const T>(h, h->L.eps),
                       ws_ptr<const T>(h, h->L.muD), ws_ptr<const T>(h, h->L.muF), mask_ptr(h),
                       tsolid_ptr(h), ws_ptr<lbm::P4<T>>(h, m1_out), m0, grid_of(h), h->tiles, ph);
}

template <int D, typename T, bool S, bool AD>
void launch_picard(const lbm_solver *h, size_t vin, size_t vout) {
    auto ph = phys_of<T>(h);
    hipLaunchKernelGGL((lbm::k_picard<D, T, S, AD>), cell_tiles(h), dim3(256), 0, h->stream,
                       ws_ptr<const lbm::P4<T>>(h, vin), ws_ptr<const lbm::P4<T>>(h, h->L.m0),
                       ws_ptr<const T>(h, h->L.eps), ws_ptr<const T>(h, h->L.muD),
                       ws_ptr<const T>(h, h->L.muF), mask_ptr(h), ws_ptr<lbm::P4<T>>(h, vout),
                       grid_of(h), h->tiles, ph, (T)h->picard_omega);
}

template <int D, typename T, bool S, bool AD>
void launch_vcorrect(const lbm_solver *h, size_t own_src, size_t m1, size_t m2_out) {
    auto ph = phys_of<T>(h);
    hipLaunchKernelGGL((lbm::k_vcorrect<D, T, S, AD>), cell_tiles(h), dim3(256), 0, h->stream,
                       ws_ptr<const lbm::P4<T>>(h, own_src), ws_ptr<const lbm::P4<T>>(h, m1),
                       ws_ptr<const T>(h, h->L.eps), mask_ptr(h), tsolid_ptr(h), tflat_ptr(h),
                       ws_ptr<lbm::P4<T>>(h, m2_out), grid_of(h), h->tiles, ph);
}

template <int D, typename T, typename P, bool S, int PH, bool AD, bool OCC>
void launch_collide_occ(const lbm_solver *h, size_t m2, size_t nbr) {
    auto ph = phys_of<T>(h);
    hipLaunchKernelGGL((lbm::k_collide<D, T, P, S, PH, AD, OCC>), cell_tiles(h), dim3(256), 0,
                       h->stream, ws_ptr<P>(h, h->L.f), ws_ptr<const lbm::P4<T>>(h, m2),
                       ws_ptr<const lbm::P4<T>>(h, nbr),
                       ws_ptr<const T>(h, h->L.eps),
                       ws_ptr<const T>(h, h->L.muD), ws_ptr<const T>(h, h->L.muF), mask_ptr(h),
                       tsolid_ptr(h), grid_of(h), h->tiles, ph);
}

// Runs with solids take the instantiation that requests the occupancy of the solid-free code
// where few of their tiles are solid-aware (lbm_solver::solid_occ).
template <int D, typename T, typename P, bool S, int PH, bool AD>
void launch_collide(const lbm_solver *h, size_t m2, size_t nbr) {
    if constexpr (S) {
        if (h->solid_occ) {
            launch_collide_occ<D, T, P, S, PH, AD, true>(h, m2, nbr);
            return;
        }
    }
    launch_collide_occ<D, T, P, S, PH, AD, false>(h, m2, nbr);
}

template <int D, typename T, typename P, bool S, int PH>
void launch_collide_vc(const lbm_solver *h, size_t m1) {
    if constexpr (D == 3 && !S)
        hipLaunchKernelGGL((lbm::k_collide_vc<T, P, PH>), dim3(8 * h->ztiles.per), dim3(lbm::ZCfg<T, P>::kThreads), 0,
                           h->stream, ws_ptr<P>(h, h->L.f), ws_ptr<const lbm::P4<T>>(h, m1),
                           ws_ptr<const T>(h, h->L.eps), ws_ptr<const T>(h, h->L.muD),
                           ws_ptr<const T>(h, h->L.muF), grid_of(h), h->ztiles, phys_of<T>(h));
}

template <int D, typename T, typename P, bool S, int PH, bool AD, bool OCC>
void launch_fused_occ(const lbm_solver *h, int prev, int next) {
    auto ph = phys_of<T>(h);
    hipLaunchKernelGGL((lbm::k_fused<D, T, P, S, PH, AD, OCC>), cell_tiles(h), dim3(256), 0, h->stream,
                       ws_ptr<P>(h, h->L.f), ws_ptr<const lbm::P4<T>>(h, h->L.m1[prev]),
                       ws_ptr<const lbm::P4<T>>(h, h->L.m2[prev]),
                       ws_ptr<lbm::P4<T>>(h, h->L.m1[next]), ws_ptr<lbm::P4<T>>(h, h->L.m2[next]),
                       ws_ptr<const T>(h, h->L.eps), ws_ptr<const T>(h, h->L.muD),
                       ws_ptr<const T>(h, h->L.muF), mask_ptr(h), tsolid_ptr(h), grid_of(h),
                       h->tiles, ph);
}

template <int D, typename T, typename P, bool S, int PH, bool AD>
void launch_fused(const lbm_solver *h, int prev, int next) {
    if constexpr (S) {
        if (h->solid_occ) {
            launch_fused_occ<D, T, P, S, PH, AD, true>(h, prev, next);
            return;
        }
    }
    launch_fused_occ<D, T, P, S, PH, AD, false>(h, prev, next);
}

template <int D, typename T, typename P, bool S, bool AD>
void launch_init(const lbm_solver *h) {
    auto ph = phys_of<T>(h);
    hipLaunchKernelGGL((lbm::k_init<D, T, P, S, AD>), cell_tiles(h), dim3(256), 0, h->stream,
                       ws_ptr<P>(h, h->L.f), ws_ptr<const lbm::P4<T>>(h, h->L.m2[0]),
                       ws_ptr<const T>(h, h->L.eps),
                       ws_ptr<const T>(h, h->L.muD), ws_ptr<const T>(h, h->L.muF), mask_ptr(h),
                       grid_of(h), h->tiles, ph);
}

template <int D, typename T, typename P, bool S, int PH, typename O>
void launch_export(const lbm_solver *h, O *out) {
    hipLaunchKernelGGL((lbm::k_export<D, T, P, S, PH, O>), cell_tiles(h), dim3(256), 0,
                       h->stream, ws_ptr<const P>(h, h->L.f), mask_ptr(h),
                       ws_ptr<const T>(h, h->L.eps), out, grid_of(h), h->tiles, phys_of<T>(h));
}

template <int D, typename T, typename P, bool S, typename I>
void launch_import(const lbm_solver *h, const I *in) {
    hipLaunchKernelGGL((lbm::k_import<D, T, P, S, I>), cell_tiles(h), dim3(256), 0, h->stream,
                       ws_ptr<P>(h, h->L.f), in, mask_ptr(h), ws_ptr<const T>(h, h->L.eps),
                       grid_of(h), h->tiles, phys_of<T>(h));
}

// Statistics blocks: one per 256 cells up to kStatsBlocks (grid-stride beyond).
inline int stats_blocks(const lbm_solver *h) {
    return (int)std::min<int64_t>(lbm::kStatsBlocks, (h->N + 255) / 256);
}

template <int D, typename T, typename P, bool S, int PH>
void launch_stats(const lbm_solver *h, size_t m2, double *part) {
    hipLaunchKernelGGL((lbm::k_stats<D, T, P, S, PH>), dim3(stats_blocks(h)), dim3(256), 0,
                       h->stream, ws_ptr<const P>(h, h->L.f), ws_ptr<const lbm::P4<T>>(h, m2),
                       ws_ptr<T>(h, h->L.vsnap), mask_ptr(h), ws_ptr<const T>(h, h->L.eps),
                       part, grid_of(h), phys_of<T>(h));
}

// ---- wet-node boundary kernels (one thread per boundary node; boundaries imply solids) -----
template <typename T>
lbm::BNodes<T> bnodes_of(const lbm_solver *h) {
    return lbm::BNodes<T>{ws_ptr<const uint32_t>(h, h->L.bcell), ws_ptr<const uint32_t>(h, h->L.bcode),
                          ws_ptr<const lbm::P4<T>>(h, h->L.bval), h->nb};
}

struct BcOutflowPass {
    static constexpr bool kDerivs = false;
    const lbm_solver *h;
    template <int D, typename T, typename P, bool S, int PH>
    void operator()() {
        if constexpr (S)
            hipLaunchKernelGGL((lbm::k_bc_outflow<D, T, P, S, PH>), flat_grid(h->nb), dim3(256), 0,
                               h->stream, ws_ptr<P>(h, h->L.f), mask_ptr(h),
                               ws_ptr<const T>(h, h->L.eps), bnodes_of<T>(h), grid_of(h),
                               phys_of<T>(h));
    }
};
struct BcRecordsPass {
    static constexpr bool kDerivs = true;
    const lbm_solver *h;
    size_t m1;
    int stage;  // 0: every node; 1: face velocity nodes again, with the viscous term
    template <int D, typename T, typename P, bool S, int PH, bool AD>
    void operator()() {
        if constexpr (S)
            hipLaunchKernelGGL((lbm::k_bc_records<D, T, P, S, PH, AD>), flat_grid(h->nb), dim3(256), 0,
                               h->stream, ws_ptr<const P>(h, h->L.f), mask_ptr(h),
                               ws_ptr<const T>(h, h->L.eps), ws_ptr<const T>(h, h->L.muD),
                               ws_ptr<const T>(h, h->L.muF), ws_ptr<lbm::P4<T>>(h, m1),
                               bnodes_of<T>(h), grid_of(h), phys_of<T>(h),
                               h->bc_rho_rule == LBM_BC_RHO_BOUNCE_BACK ? 1 : 0, stage);
    }
};
struct BcFixPass {
    static constexpr bool kDerivs = false;
    const lbm_solver *h;
    size_t m1, m2;
    template <int D, typename T, typename P, bool S, int PH>
    void operator()() {
        if constexpr (S)
            hipLaunchKernelGGL((lbm::k_bc_fix<T>), flat_grid(h->nb), dim3(256), 0, h->stream,
                               ws_ptr<const lbm::P4<T>>(h, m1), ws_ptr<lbm::P4<T>>(h, m2),
                               bnodes_of<T>(h));
    }
};
struct BcRebuildPass {  // own records m2, stencil neighbours' nbr
    static constexpr bool kDerivs = true;
    const lbm_solver *h;
    size_t m2, nbr;
    template <int D, typename T, typename P, bool S, int PH, bool AD>
    void operator()() {
        if constexpr (S)
            hipLaunchKernelGGL((lbm::k_bc_rebuild<D, T, P, S, PH, AD>), flat_grid(h->nb), dim3(256), 0,
                               h->stream, ws_ptr<P>(h, h->L.f), ws_ptr<const lbm::P4<T>>(h, m2),
                               ws_ptr<const lbm::P4<T>>(h, nbr),
                               ws_ptr<const T>(h, h->L.eps), ws_ptr<const T>(h, h->L.muD),
                               ws_ptr<const T>(h, h->L.muF), mask_ptr(h), bnodes_of<T>(h),
                               grid_of(h), phys_of<T>(h), h->bc_scheme);
    }
};

// Runs one pass for the handle's configuration: fn.template operator()<D, T, P, S, PH>(), with
// the derivative source AD appended for passes that read porosity derivatives (kDerivs).
template <typename F, int D, typename T, typename P, bool S, int PH, bool AD>
inline void call_pass(F &fn) {
    if constexpr (F::kDerivs) fn.template operator()<D, T, P, S, PH, AD>();
    else fn.template operator()<D, T, P, S, PH>();
}

template <bool AD, typename F>
void dispatch_cfg(const lbm_solver *h, F &fn) {
    const bool s = h->solids;
    const int ph = h->phase;
#define LBM_DISPATCH_T(DD, TT, PP)                                   \
    if (s) {                                                         \
        if (ph) call_pass<F, DD, TT, PP, true, 1, AD>(fn);           \
        else call_pass<F, DD, TT, PP, true, 0, AD>(fn);              \
    } else {                                                         \
        if (ph) call_pass<F, DD, TT, PP, false, 1, AD>(fn);          \
        else call_pass<F, DD, TT, PP, false, 0, AD>(fn);             \
    }
#define LBM_DISPATCH_D(DD)                                                        \
    switch (h->storage) {                                                         \
    case LBM_F64: { LBM_DISPATCH_T(DD, double, double) } break;                   \
    case LBM_F32: { LBM_DISPATCH_T(DD, float, float) } break;                     \
    case LBM_F16_SHIFTED: { LBM_DISPATCH_T(DD, float, _Float16) } break;          \
    default: { LBM_DISPATCH_T(DD, float, __bf16) } break;                         \
    }
    if (h->D == 2) { LBM_DISPATCH_D(2) }
    else { LBM_DISPATCH_D(3) }
#undef LBM_DISPATCH_D
#undef LBM_DISPATCH_T
}

// The kernels that read analytic porosity derivatives are instantiated in a translation unit
// of their own (lbm_analytic.hip), compiled in parallel with this one.
template <typename F>
void dispatch_analytic(const lbm_solver *h, F &fn);

template <typename F>
void dispatch(const lbm_solver *h, F &&fn) {
    using G = std::decay_t<F>;
    if constexpr (G::kDerivs) {
        if (h->analytic) {
            dispatch_analytic<G>(h, fn);
            return;
        }
    }
    dispatch_cfg<false>(h, fn);
}

struct MomentsPass {
    static constexpr bool kDerivs = true;
    const lbm_solver *h;
    size_t m1_out;
    template <int D, typename T, typename P, bool S, int PH, bool AD>
    void operator()() { launch_moments<D, T, P, S, PH, AD>(h, m1_out); }
};
struct VcorrectPass {
    static constexpr bool kDerivs = true;
    const lbm_solver *h;
    size_t own_src, m1, m2_out;
    template <int D, typename T, typename P, bool S, int PH, bool AD>
    void operator()() { launch_vcorrect<D, T, S, AD>(h, own_src, m1, m2_out); }
};
struct CollidePass {  // own records m2, stencil neighbours' nbr (= m2 in the two-pass scheme)
    static constexpr bool kDerivs = true;
    const lbm_solver *h;
    size_t m2, nbr;
    template <int D, typename T, typename P, bool S, int PH, bool AD>
    void operator()() { launch_collide<D, T, P, S, PH, AD>(h, m2, nbr); }
};
struct CollideVcPass {  // only dispatched for runs with fused_vc (D3Q27, no solids)
    static constexpr bool kDerivs = false;
    const lbm_solver *h;
    size_t m1;
    template <int D, typename T, typename P, bool S, int PH>
    void operator()() { launch_collide_vc<D, T, P, S, PH>(h, m1); }
};
struct PicardPass {
    static constexpr bool kDerivs = true;
    const lbm_solver *h;
    size_t vin, vout;
    template <int D, typename T, typename P, bool S, int PH, bool AD>
    void operator()() { launch_picard<D, T, S, AD>(h, vin, vout); }
};
struct FusedPass {
    static constexpr bool kDerivs = true;
    const lbm_solver *h;
    int prev, next;
    template <int D, typename T, typename P, bool S, int PH, bool AD>
    void operator()() { launch_fused<D, T, P, S, PH, AD>(h, prev, next); }
};
struct InitPass {
    static constexpr bool kDerivs = true;
    const lbm_solver *h;
    template <int D, typename T, typename P, bool S, int PH, bool AD>
    void operator()() { launch_init<D, T, P, S, AD>(h); }
};
struct StatsPass {
    static constexpr bool kDerivs = false;
    const lbm_solver *h;
    size_t m2;
    double *part;  // per-block partial sums (stats_blocks(h) rows of kStatsSlots)
    template <int D, typename T, typename P, bool S, int PH>
    void operator()() { launch_stats<D, T, P, S, PH>(h, m2, part); }
};
struct ExportPass {
    static constexpr bool kDerivs = false;
    const lbm_solver *h;
    void *out;
    int dtype;
    template <int D, typename T, typename P, bool S, int PH>
    void operator()() {
        if (dtype == LBM_DTYPE_F64) launch_export<D, T, P, S, PH, double>(h, (double *)out);
        else launch_export<D, T, P, S, PH, float>(h, (float *)out);
    }
};
struct ImportPass {
    static constexpr bool kDerivs = false;
    const lbm_solver *h;
    const void *in;
    int dtype;
    template <int D, typename T, typename P, bool S, int PH>
    void operator()() {
        if (dtype == LBM_DTYPE_F64) launch_import<D, T, P, S, double>(h, (const double *)in);
        else launch_import<D, T, P, S, float>(h, (const float *)in);
    }
};


}  // namespace lbmh
