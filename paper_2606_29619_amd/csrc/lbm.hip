// lbm.hip -- C ABI (include/lbm.h) of the gfx950 porous-media lattice Boltzmann library.
//
// Host side: argument validation, workspace layout, uploads and kernel dispatch.  All device
// memory comes from the caller's workspace; all work goes to the caller's stream.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include "lbm_bc.hpp"
#include "lbm_device.hpp"
#include "lbm_host.hpp"
#include "lbm_launch.hpp"

namespace lbmh {

// Velocity of the two-pass step after the one-shot correction into m2: the boundary records,
// then the Picard iterations (App. F), each followed by the boundary records again.  Returns
// the buffer that holds the final (rho, v) records.
size_t velocity_stage(lbm_solver *h, size_t m1, size_t m2) {
    if (h->bc_vp) dispatch(h, BcFixPass{h, m1, m2});
    size_t a = m2, b = h->L.mx;
    for (int k = 0; k < h->picard_iters; ++k) {
        dispatch(h, PicardPass{h, a, b});
        if (h->bc_vp) dispatch(h, BcFixPass{h, m1, b});
        std::swap(a, b);
    }
    return a;
}

// Boundary records over the bulk moments in m1: every node, then the face velocity nodes
// again with the viscous term of their wall-normal acceleration.
void boundary_records(lbm_solver *h, size_t m1) {
    if (!h->bc_vp) return;
    dispatch(h, BcRecordsPass{h, m1, 0});
    if (h->bc_visc) dispatch(h, BcRecordsPass{h, m1, 1});
}

// Moments of the current state into internal packed records; returns the offset of the
// (rho, v) records.  Under the lagged scheme with a valid history the correction takes its
// neighbour values from the previous step's records, which stay untouched; wet-node
// boundaries take their outflow copies and records as in the two-pass scheme.
size_t current_moments(lbm_solver *h) {
    if (h->scheme == LBM_SCHEME_LAGGED && h->have_prev) {
        const int nx = h->cur ^ 1;
        if (h->bc_outflow) dispatch(h, BcOutflowPass{h});
        dispatch(h, MomentsPass{h, h->L.m1[nx]});
        boundary_records(h, h->L.m1[nx]);
        dispatch(h, VcorrectPass{h, h->L.m1[nx], h->L.m1[h->cur], h->L.m2[nx]});
        if (h->bc_vp) dispatch(h, BcFixPass{h, h->L.m1[nx], h->L.m2[nx]});
        return h->L.m2[nx];
    }
    const int c = h->cur;
    if (h->bc_outflow) dispatch(h, BcOutflowPass{h});
    dispatch(h, MomentsPass{h, h->L.m1[c]});
    boundary_records(h, h->L.m1[c]);
    dispatch(h, VcorrectPass{h, h->L.m1[c], h->L.m1[c], h->L.m2[c]});
    return velocity_stage(h, h->L.m1[c], h->L.m2[c]);
}

// Enqueue one time step; ev (optional) receives events after each kernel class.
hipError_t one_step(lbm_solver *h, hipEvent_t *ev) {
    hipError_t e = hipSuccess;
    if (h->scheme == LBM_SCHEME_LAGGED && h->have_prev) {
        const int nx = h->cur ^ 1;
        if (h->nb) {
            // wet-node boundaries: the lagged step as separate passes around the boundary
            // kernels; the correction, the boundary rebuild and the collision take their
            // neighbours' records from the previous step (m1 / m2 of pair cur)
            if (h->bc_outflow) dispatch(h, BcOutflowPass{h});
            dispatch(h, MomentsPass{h, h->L.m1[nx]});
            boundary_records(h, h->L.m1[nx]);
            if (ev) e = hipEventRecord(ev[0], h->stream);
            dispatch(h, VcorrectPass{h, h->L.m1[nx], h->L.m1[h->cur], h->L.m2[nx]});
            if (h->bc_vp) dispatch(h, BcFixPass{h, h->L.m1[nx], h->L.m2[nx]});
            if (ev && e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
            if (h->bc_vp) dispatch(h, BcRebuildPass{h, h->L.m2[nx], h->L.m2[h->cur]});
            dispatch(h, CollidePass{h, h->L.m2[nx], h->L.m2[h->cur]});
            if (ev && e == hipSuccess) e = hipEventRecord(ev[2], h->stream);
        } else {
            if (ev) e = hipEventRecord(ev[0], h->stream);
            if (ev && e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
            dispatch(h, FusedPass{h, h->cur, nx});
            if (ev && e == hipSuccess) e = hipEventRecord(ev[2], h->stream);
        }
        h->cur = nx;
    } else {
        const int c = h->cur;
        if (h->fused_vc) {
            // velocity correction inside the collision pass (timed with it)
            dispatch(h, MomentsPass{h, h->L.m1[c]});
            if (ev) e = hipEventRecord(ev[0], h->stream);
            if (ev && e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
            dispatch(h, CollideVcPass{h, h->L.m1[c]});
            if (ev && e == hipSuccess) e = hipEventRecord(ev[2], h->stream);
            h->have_prev = true;
            if (e == hipSuccess) e = hipGetLastError();
            h->phase ^= 1;
            h->step += 1;
            return e;
        }
        // wet-node boundaries: outflow copies, boundary records and population rebuild around
        // the bulk passes (they are timed with the pass they follow)
        if (h->bc_outflow) dispatch(h, BcOutflowPass{h});
        dispatch(h, MomentsPass{h, h->L.m1[c]});
        boundary_records(h, h->L.m1[c]);
        if (ev) e = hipEventRecord(ev[0], h->stream);
        dispatch(h, VcorrectPass{h, h->L.m1[c], h->L.m1[c], h->L.m2[c]});
        const size_t mv = velocity_stage(h, h->L.m1[c], h->L.m2[c]);
        if (ev && e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
        if (h->bc_vp) dispatch(h, BcRebuildPass{h, mv, mv});
        dispatch(h, CollidePass{h, mv, mv});
        if (ev && e == hipSuccess) e = hipEventRecord(ev[2], h->stream);
        h->have_prev = true;  // this step's records are the next step's history
    }
    if (e == hipSuccess) e = hipGetLastError();
    h->phase ^= 1;
    h->step += 1;
    return e;
}

int check_handle(const lbm_solver *h) {
    if (!h) return fail(LBM_ERR_INVALID_ARG, "null solver handle");
    if (!h->ws) return fail(LBM_ERR_STATE, "solver handle is not initialised");
    return LBM_OK;
}

// Packed-row tiles, unless the caller asks for rectangular tiles: always for FP32 / FP64
// storage; for the 16-bit forms, whose moment and lagged passes then read the porosity of their
// decode through the caches (the 26 neighbours of a D3Q27 cell) instead of from LDS, only on
// D3Q27 runs whose rectangular tiles would leave at least 30 % of the lanes idle.  Measured on
// the first 12 requests of the serving stream (FP16, packed against rectangular MLUPS): x
// extents 81, 37, 159 (37-42 % idle) +8 %, +3 %, +12 %; 107, 125, 50 (2-22 % idle) -14 %,
// -16 %, -10 %; D2Q9 rows of 291 and 350 cells (43 %, 32 %) -9 %, -4 %.
bool packed_rows_ok(const lbm_params *p) {
    if (p->tiles == LBM_TILES_RECTANGULAR) return false;
    if (p->storage == LBM_F32 || p->storage == LBM_F64) return true;
    const int tx = rect_tile_x(p->nx);
    const int padded = (p->nx + tx - 1) / tx * tx;
    return p->lattice == LBM_D3Q27 && 10 * (padded - p->nx) >= 3 * padded;
}

int validate_shape(const lbm_params *p, int *D, int *Q, size_t *sp, size_t *s, int64_t *N) {
    if (!p) return fail(LBM_ERR_INVALID_ARG, "params is NULL");
    if (p->lattice == LBM_D2Q9) { *D = 2; *Q = 9; }
    else if (p->lattice == LBM_D3Q27) { *D = 3; *Q = 27; }
    else return fail(LBM_ERR_INVALID_ARG, "lattice must be LBM_D2Q9 or LBM_D3Q27, got %d", p->lattice);
    if (p->storage == LBM_F64) { *sp = 8; *s = 8; }
    else if (p->storage == LBM_F32) { *sp = 4; *s = 4; }
    else if (p->storage == LBM_F16_SHIFTED || p->storage == LBM_BF16_SHIFTED) { *sp = 2; *s = 4; }
    else return fail(LBM_ERR_UNSUPPORTED, "storage %d is not supported", p->storage);
    if (p->shift != LBM_SHIFT_WEIGHTS && p->shift != LBM_SHIFT_POROUS)
        return fail(LBM_ERR_INVALID_ARG, "shift must be LBM_SHIFT_WEIGHTS or LBM_SHIFT_POROUS, got %d", p->shift);
    if (p->scheme != LBM_SCHEME_TWO_PASS && p->scheme != LBM_SCHEME_LAGGED)
        return fail(LBM_ERR_INVALID_ARG, "scheme must be LBM_SCHEME_TWO_PASS or LBM_SCHEME_LAGGED, got %d", p->scheme);
    if (p->picard_iters < 0 || p->picard_iters > 64)
        return fail(LBM_ERR_INVALID_ARG, "picard_iters must be in 0..64, got %d", p->picard_iters);
    if (p->picard_iters && !(p->picard_omega > 0.0 && p->picard_omega <= 1.0))
        return fail(LBM_ERR_INVALID_ARG, "picard_omega must be in (0, 1]");
    if (p->picard_iters && p->scheme != LBM_SCHEME_TWO_PASS)
        return fail(LBM_ERR_UNSUPPORTED, "Picard iterations need LBM_SCHEME_TWO_PASS");
    if ((p->grad_eps == nullptr) != (p->hess_eps == nullptr))
        return fail(LBM_ERR_INVALID_ARG, "grad_eps and hess_eps go together (both or neither)");
    if (p->tiles != LBM_TILES_AUTO && p->tiles != LBM_TILES_RECTANGULAR)
        return fail(LBM_ERR_INVALID_ARG, "tiles must be LBM_TILES_AUTO or LBM_TILES_RECTANGULAR, got %d", p->tiles);
    if (p->passes != LBM_PASSES_AUTO && p->passes != LBM_PASSES_SEPARATE && p->passes != LBM_PASSES_FUSED)
        return fail(LBM_ERR_INVALID_ARG, "passes must be LBM_PASSES_AUTO, _SEPARATE or _FUSED, got %d", p->passes);
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(LBM_ERR_INVALID_ARG, "dimensions must be >= 1 (got %d x %d x %d)", p->nx, p->ny, p->nz);
    if (*D == 2 && p->nz != 1) return fail(LBM_ERR_INVALID_ARG, "D2Q9 needs nz = 1 (got %d)", p->nz);
    if (p->ny > 4 * 65535 || p->nz > 65535)
        return fail(LBM_ERR_UNSUPPORTED, "ny must be <= 262140 and nz <= 65535");
    *N = (int64_t)p->nx * p->ny * p->nz;
    // every array plane is addressed with 32-bit byte offsets; the largest plane is the packed
    // moment record field, four values per cell
    if ((uint64_t)*N * 4 * *s >= ((uint64_t)1 << 32))
        return fail(LBM_ERR_UNSUPPORTED, "%lld cells of 4 x %zu-byte moment records exceed 4 GiB",
                    (long long)*N, *s);
    return LBM_OK;
}

// Outward normal(s) of a bc_normal code (LBM_NORMAL_* or LBM_NORMAL_AXES) as one entry per axis
// in {-1, 0, 1}; returns their number, or -1 for a code that is not one of those.
int decode_normal(int code, int D, int nv[3]) {
    nv[0] = nv[1] = nv[2] = 0;
    if (code >= 0 && code < 2 * D) {
        nv[code >> 1] = (code & 1) ? 1 : -1;
        return 1;
    }
    if (code < 64 || code >= 128) return -1;
    int k = 0;
    for (int a = 0; a < 3; ++a) {
        const int sa = ((code - 64) >> (2 * a)) & 3;
        if (sa == 3 || (sa != 0 && a >= D)) return -1;
        nv[a] = sa == 1 ? -1 : (sa == 2 ? 1 : 0);
        k += nv[a] != 0 ? 1 : 0;
    }
    return k > 0 ? k : -1;
}

// The normal code the kernels use: 0..5 for one normal, 64 + fields for two or three.
uint32_t canonical_normal(const int nv[3]) {
    int k = 0, a1 = 0;
    uint32_t c = 64;
    for (int a = 0; a < 3; ++a)
        if (nv[a] != 0) {
            ++k;
            a1 = a;
            c += (uint32_t)(nv[a] < 0 ? 1 : 2) << (2 * a);
        }
    return k == 1 ? (uint32_t)(2 * a1 + (nv[a1] > 0 ? 1 : 0)) : c;
}

// Boundary nodes of a run: validates them and returns their count (host only); visc: some face
// velocity node takes its density from mass continuity (the viscous term then needs a stage).
int boundary_nodes(const lbm_params *p, int D, int64_t N, uint32_t *count, bool *outflow,
                   bool *vp, bool *visc) {
    *count = 0;
    *outflow = *vp = *visc = false;
    if (!p->bc_type) return LBM_OK;
    if (p->bc_scheme < LBM_BC_EQUILIBRIUM || p->bc_scheme > LBM_BC_TMS)
        return fail(LBM_ERR_INVALID_ARG, "bad bc_scheme %d", p->bc_scheme);
    if (p->bc_rho_rule != LBM_BC_RHO_CONTINUITY && p->bc_rho_rule != LBM_BC_RHO_BOUNCE_BACK)
        return fail(LBM_ERR_INVALID_ARG, "bad bc_rho_rule %d", p->bc_rho_rule);
    if (!p->bc_normal) return fail(LBM_ERR_INVALID_ARG, "bc_normal is required with bc_type");
    if (!p->mask) return fail(LBM_ERR_INVALID_ARG, "wet-node boundaries need solid cells (mask)");
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    auto cell = [&](int x, int y, int z) {
        x = (x % nx + nx) % nx;
        y = (y % ny + ny) % ny;
        z = (z % nz + nz) % nz;
        return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
    };
    auto bulk = [&](int64_t c) { return !p->mask[c] && p->bc_type[c] == LBM_NODE_BULK; };
    uint32_t k = 0;
    for (int64_t n = 0; n < N; ++n) {
        const int t = p->bc_type[n];
        if (t == LBM_NODE_BULK) continue;
        if (t > LBM_NODE_OUTFLOW) return fail(LBM_ERR_INVALID_ARG, "bc_type[%lld] = %d", (long long)n, t);
        int o[3];
        const int nn = decode_normal(p->bc_normal[n], D, o);
        if (nn < 0) return fail(LBM_ERR_INVALID_ARG, "bc_normal[%lld] = %d", (long long)n, p->bc_normal[n]);
        if (p->mask[n]) return fail(LBM_ERR_INVALID_ARG, "boundary node %lld is solid", (long long)n);
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        for (int a = 0; a < 3; ++a) {
            if (o[a] == 0) continue;
            const int64_t out = cell(x + (a == 0 ? o[0] : 0), y + (a == 1 ? o[1] : 0), z + (a == 2 ? o[2] : 0));
            if (!p->mask[out])
                return fail(LBM_ERR_INVALID_ARG, "the outward neighbour of boundary node %lld along axis %d must be solid", (long long)n, a);
        }
        if (nn == 1) {
            if (!bulk(cell(x - o[0], y - o[1], z - o[2])))
                return fail(LBM_ERR_INVALID_ARG, "the inward neighbour of boundary node %lld must be a bulk fluid cell", (long long)n);
        } else {
            if (t != LBM_NODE_VELOCITY)
                return fail(LBM_ERR_INVALID_ARG, "edge or corner node %lld must be a velocity node", (long long)n);
            if (!bulk(cell(x - o[0], y - o[1], z - o[2])) || !bulk(cell(x - 2 * o[0], y - 2 * o[1], z - 2 * o[2])))
                return fail(LBM_ERR_INVALID_ARG, "edge or corner node %lld needs two bulk fluid cells along its inward diagonal", (long long)n);
        }
        if (t == LBM_NODE_VELOCITY && p->bc_velocity)
            for (int a = 0; a < D; ++a)
                if (!is_finite(p->bc_velocity[(int64_t)a * N + n]))
                    return fail(LBM_ERR_INVALID_ARG, "bc_velocity must be finite");
        if (t == LBM_NODE_PRESSURE && p->bc_density && !(is_finite(p->bc_density[n]) && p->bc_density[n] > 0))
            return fail(LBM_ERR_INVALID_ARG, "bc_density[%lld] must be finite and > 0", (long long)n);
        if (t == LBM_NODE_OUTFLOW) *outflow = true;
        else *vp = true;
        if (t == LBM_NODE_VELOCITY && nn == 1 && p->bc_rho_rule == LBM_BC_RHO_CONTINUITY) *visc = true;
        ++k;
    }
    *count = k;
    return LBM_OK;
}

int enqueue_stats(lbm_solver *h, double *part, double *res) {
    const size_t m2 = current_moments(h);
    LAUNCH_CHECK();
    dispatch(h, StatsPass{h, m2, part});
    LAUNCH_CHECK();
    hipLaunchKernelGGL(lbm::k_stats_final, dim3(1), dim3(256), 0, h->stream, part,
                       stats_blocks(h), res);
    LAUNCH_CHECK();
    return LBM_OK;
}

// ---- statistics without allocation ---------------------------------------------------------
// Per-block partial sums of lbm_stats_noalloc: at most kStatsBlocks rows of kStatsSlots doubles
// (64 KiB).  Every GPU the library runs on holds its own copy until the process ends.  In host
// code the name stands for no device address: kernels get the pointer that hipGetSymbolAddress
// returns for the device, looked up once per device and kept.
static __device__ __align__(256) double scratch[lbm::kStatsBlocks * lbm::kStatsSlots];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

int scratch_of_device(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LBM_ERR_UNSUPPORTED, "device %d is beyond the %d devices the statistics "
                    "scratch serves", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) HIP_TRY(hipSetDevice(cur));
        if (e != hipSuccess)
            return fail(LBM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace lbmh

using namespace lbmh;

extern "C" {

LBM_API const char *lbm_last_error(void) { return g_err.c_str(); }

LBM_API int lbm_lattice_info(int lattice, int *c_out, int *opp_out) {
    if (!c_out || !opp_out) return fail(LBM_ERR_INVALID_ARG, "null output pointer");
    if (lattice == LBM_D2Q9) {
        for (int i = 0; i < 9; ++i) {
            for (int a = 0; a < 3; ++a) c_out[3 * i + a] = lbm::Lat<2>::c[i][a];
            opp_out[i] = lbm::Lat<2>::opp[i];
        }
        return 9;
    }
    if (lattice == LBM_D3Q27) {
        for (int i = 0; i < 27; ++i) {
            for (int a = 0; a < 3; ++a) c_out[3 * i + a] = lbm::Lat<3>::c[i][a];
            opp_out[i] = lbm::Lat<3>::opp[i];
        }
        return 27;
    }
    return fail(LBM_ERR_INVALID_ARG, "unknown lattice %d", lattice);
}

LBM_API int lbm_footprint(const lbm_params *p, size_t *workspace_bytes) {
    int D, Q;
    size_t sp, s;
    int64_t N;
    if (!workspace_bytes) return fail(LBM_ERR_INVALID_ARG, "workspace_bytes is NULL");
    int rc = validate_shape(p, &D, &Q, &sp, &s, &N);
    if (rc) return rc;
    uint32_t nb = 0;
    bool bo, bv, bvisc;
    rc = boundary_nodes(p, D, N, &nb, &bo, &bv, &bvisc);
    if (rc) return rc;
    const lbm::Tiling tl = make_tiling(p->nx, p->ny, p->nz, packed_rows_ok(p));
    *workspace_bytes = make_layout(Q, D, (size_t)N, sp, s, p->mask != nullptr,
                                   p->scheme == LBM_SCHEME_LAGGED, 8 * (size_t)tl.per, nb,
                                   p->picard_iters > 0, p->grad_eps != nullptr).total;
    return LBM_OK;
}

LBM_API int lbm_create(const lbm_params *p, void *dev_workspace, size_t workspace_bytes,
                       void *hip_stream, lbm_solver **out) {
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int D, Q;
    size_t sp, s;
    int64_t N;
    int rc = validate_shape(p, &D, &Q, &sp, &s, &N);
    if (rc) return rc;
    if (!(is_finite(p->RT) && p->RT > 0)) return fail(LBM_ERR_INVALID_ARG, "RT must be finite and > 0");
    if (!(is_finite(p->nu_f) && p->nu_f >= 0)) return fail(LBM_ERR_INVALID_ARG, "nu_f must be finite and >= 0");
    if (!(is_finite(p->nu_eff_ref) && p->nu_eff_ref > 0))
        return fail(LBM_ERR_INVALID_ARG, "nu_eff_ref must be finite and > 0");
    if (p->nu_eff_pow < -1 || p->nu_eff_pow > 1) return fail(LBM_ERR_INVALID_ARG, "nu_eff_pow must be -1, 0 or 1");
    if (!std::isnan(p->eta_eff) && !(is_finite(p->eta_eff) && p->eta_eff >= 0))
        return fail(LBM_ERR_INVALID_ARG, "eta_eff must be NaN or finite and >= 0");
    for (int a = 0; a < 3; ++a)
        if (!is_finite(p->b[a])) return fail(LBM_ERR_INVALID_ARG, "body force must be finite");
    if (!(is_finite(p->rho0) && p->rho0 > 0)) return fail(LBM_ERR_INVALID_ARG, "rho0 must be finite and > 0");
    if (!p->eps || !p->kappa || !p->forch) return fail(LBM_ERR_INVALID_ARG, "eps, kappa and forch are required");
    bool any_fluid = false;
    for (int64_t n = 0; n < N; ++n) {
        const double e = p->eps[n];
        if (!(e > 0.0 && e <= 1.0)) return fail(LBM_ERR_INVALID_ARG, "eps[%lld] = %g is outside (0, 1]", (long long)n, e);
        const bool solid = p->mask && p->mask[n];
        if (p->mask && p->mask[n] > 1) return fail(LBM_ERR_INVALID_ARG, "mask[%lld] must be 0 or 1", (long long)n);
        if (solid) continue;
        any_fluid = true;
        const double k = p->kappa[n], c = p->forch[n];
        if (!(k > 0.0)) return fail(LBM_ERR_INVALID_ARG, "kappa[%lld] = %g must be > 0 (or +inf)", (long long)n, k);
        if (!(is_finite(c) && c >= 0.0)) return fail(LBM_ERR_INVALID_ARG, "forch[%lld] = %g must be finite and >= 0", (long long)n, c);
        if (p->rho_init && !(is_finite(p->rho_init[n]) && p->rho_init[n] > 0))
            return fail(LBM_ERR_INVALID_ARG, "rho_init[%lld] must be finite and > 0", (long long)n);
        if (p->v_init)
            for (int a = 0; a < D; ++a)
                if (!is_finite(p->v_init[(int64_t)a * N + n]))
                    return fail(LBM_ERR_INVALID_ARG, "v_init must be finite");
        if (p->grad_eps) {
            for (int a = 0; a < D; ++a)
                if (!is_finite(p->grad_eps[(int64_t)a * N + n]))
                    return fail(LBM_ERR_INVALID_ARG, "grad_eps must be finite on fluid cells");
            for (int j = 0; j < D * (D + 1) / 2; ++j)
                if (!is_finite(p->hess_eps[(int64_t)j * N + n]))
                    return fail(LBM_ERR_INVALID_ARG, "hess_eps must be finite on fluid cells");
        }
    }
    if (!any_fluid) return fail(LBM_ERR_INVALID_ARG, "no fluid cell");
    const bool solids = p->mask != nullptr;
    uint32_t nb = 0;
    bool bc_outflow = false, bc_vp = false, bc_visc = false;
    rc = boundary_nodes(p, D, N, &nb, &bc_outflow, &bc_vp, &bc_visc);
    if (rc) return rc;
    const lbm::Tiling tiles = make_tiling(p->nx, p->ny, p->nz, packed_rows_ok(p));
    const Layout L = make_layout(Q, D, (size_t)N, sp, s, solids, p->scheme == LBM_SCHEME_LAGGED,
                                 8 * (size_t)tiles.per, nb, p->picard_iters > 0,
                                 p->grad_eps != nullptr);
    if (!dev_workspace) return fail(LBM_ERR_INVALID_ARG, "dev_workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256)
        return fail(LBM_ERR_WORKSPACE, "dev_workspace must be 256-byte aligned");
    if (workspace_bytes < L.total)
        return fail(LBM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes needed",
                    workspace_bytes, L.total);

    lbm_solver *h = new (std::nothrow) lbm_solver();
    if (!h) return fail(LBM_ERR_INVALID_ARG, "out of host memory");
    h->lattice = p->lattice;
    h->D = D;
    h->Q = Q;
    h->storage = p->storage;
    h->nx = p->nx; h->ny = p->ny; h->nz = p->nz;
    h->N = N;
    h->solids = solids;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->ws = reinterpret_cast<char *>(dev_workspace);
    h->L = L;
    h->tiles = tiles;
    h->step = 0;
    h->phase = 0;
    h->scheme = p->scheme;
    h->cur = 0;
    h->have_prev = true;  // the initial fields stand for the previous step
    h->RT = p->RT;
    h->nu_f = p->nu_f;
    h->nu_eff_ref = p->nu_eff_ref;
    h->nu_eff_pow = p->nu_eff_pow;
    h->eta_eff = p->eta_eff;
    h->rho0 = p->rho0;
    h->shift = p->shift;
    h->nb = nb;
    h->bc_outflow = bc_outflow;
    h->bc_vp = bc_vp;
    h->bc_visc = bc_visc;
    h->bc_scheme = p->bc_scheme;
    h->bc_rho_rule = p->bc_rho_rule;
    h->picard_iters = p->picard_iters;
    h->picard_omega = p->picard_omega;
    h->analytic = p->grad_eps != nullptr;
    {
        // the fused correction-collision kernel: D3Q27, any storage, no solids, wet nodes,
        // Picard iterations or analytic derivatives, whole tiles; AUTO takes
        // it where the chunks are at least 16 planes long (shorter ones correct and stage too
        // many end planes again)
        const bool half = p->storage == LBM_F16_SHIFTED || p->storage == LBM_BF16_SHIFTED;
        const int tx = p->storage == LBM_F64 ? lbm::ZCfg<double>::kX
                       : half               ? lbm::ZCfg<float, _Float16>::kX
                                            : lbm::ZCfg<float>::kX;
        const int ty = p->storage == LBM_F64 ? lbm::ZCfg<double>::kY
                       : half               ? lbm::ZCfg<float, _Float16>::kY
                                            : lbm::ZCfg<float>::kY;
        const bool able = D == 3 && !solids &&
                          nb == 0 && p->picard_iters == 0 && !h->analytic &&
                          p->scheme == LBM_SCHEME_TWO_PASS && p->nx % tx == 0 && p->ny % ty == 0;
        if (able) h->ztiles = make_ztiling(p->nx, p->ny, p->nz, tx, ty);
        h->fused_vc = able && (p->passes == LBM_PASSES_FUSED ||
                               (p->passes == LBM_PASSES_AUTO && h->ztiles.zc >= 16));
    }
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(LBM_ERR_HIP, "hipGetDevice failed");
    }
    for (int a = 0; a < 3; ++a) h->b[a] = a < D ? p->b[a] : 0.0;

    auto cleanup = [&](int code) {
        delete h;
        return code;
    };
    // Stage the FP64 input fields in the population region (sized for 4 FP64 arrays), derive
    // the static fields, then stage the initial moments the same way.
    const size_t NB = (size_t)N * sizeof(double);
    double *st = ws_ptr<double>(h, L.f);
    hipError_t e;
    if ((e = hipMemcpyAsync(st, p->eps, NB, hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(st + N, p->kappa, NB, hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(st + 2 * N, p->forch, NB, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
        return cleanup(fail(LBM_ERR_HIP, "upload of input fields failed: %s", hipGetErrorString(e)));
    if (solids && (e = hipMemcpyAsync(h->ws + L.mask, p->mask, (size_t)N, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
        return cleanup(fail(LBM_ERR_HIP, "upload of mask failed: %s", hipGetErrorString(e)));
    if (solids) {
        uint8_t *ts = reinterpret_cast<uint8_t *>(h->ws + L.tsolid);
        // padding workgroups past the last tile write no flag
        if ((e = hipMemsetAsync(ts, 0, 8 * (size_t)h->tiles.per, h->stream)) != hipSuccess)
            return cleanup(fail(LBM_ERR_HIP, "tile-flag clear failed: %s", hipGetErrorString(e)));
        if (D == 2) hipLaunchKernelGGL(lbm::k_tile_solid<2>, cell_tiles(h), dim3(256), 0, h->stream, mask_ptr(h), grid_of(h), h->tiles, ts);
        else hipLaunchKernelGGL(lbm::k_tile_solid<3>, cell_tiles(h), dim3(256), 0, h->stream, mask_ptr(h), grid_of(h), h->tiles, ts);
        if ((e = hipGetLastError()) != hipSuccess)
            return cleanup(fail(LBM_ERR_HIP, "tile-flag kernel failed: %s", hipGetErrorString(e)));
    }
    if (h->storage == LBM_F64)
        hipLaunchKernelGGL(lbm::k_static<double>, flat_grid(N), dim3(256), 0, h->stream, st, st + N, st + 2 * N,
                           ws_ptr<double>(h, L.eps), ws_ptr<double>(h, L.muD), ws_ptr<double>(h, L.muF), N, p->nu_f);
    else
        hipLaunchKernelGGL(lbm::k_static<float>, flat_grid(N), dim3(256), 0, h->stream, st, st + N, st + 2 * N,
                           ws_ptr<float>(h, L.eps), ws_ptr<float>(h, L.muD), ws_ptr<float>(h, L.muF), N, p->nu_f);
    if ((e = hipGetLastError()) != hipSuccess)
        return cleanup(fail(LBM_ERR_HIP, "static-field kernel failed: %s", hipGetErrorString(e)));
    if (!h->analytic) {  // after the static-field kernel has written eps (same stream)
        uint8_t *tf = reinterpret_cast<uint8_t *>(h->ws + L.tflat);
        if (h->storage == LBM_F64) {
            if (D == 2) hipLaunchKernelGGL((lbm::k_tile_flat<2, double>), cell_tiles(h), dim3(256), 0, h->stream, ws_ptr<const double>(h, L.eps), grid_of(h), h->tiles, tf);
            else hipLaunchKernelGGL((lbm::k_tile_flat<3, double>), cell_tiles(h), dim3(256), 0, h->stream, ws_ptr<const double>(h, L.eps), grid_of(h), h->tiles, tf);
        } else {
            if (D == 2) hipLaunchKernelGGL((lbm::k_tile_flat<2, float>), cell_tiles(h), dim3(256), 0, h->stream, ws_ptr<const float>(h, L.eps), grid_of(h), h->tiles, tf);
            else hipLaunchKernelGGL((lbm::k_tile_flat<3, float>), cell_tiles(h), dim3(256), 0, h->stream, ws_ptr<const float>(h, L.eps), grid_of(h), h->tiles, tf);
        }
        if ((e = hipGetLastError()) != hipSuccess)
            return cleanup(fail(LBM_ERR_HIP, "flat-tile kernel failed: %s", hipGetErrorString(e)));
    }
    const double *rho_st = nullptr, *v_st = nullptr;
    if (p->rho_init) {
        if ((e = hipMemcpyAsync(st, p->rho_init, NB, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
            return cleanup(fail(LBM_ERR_HIP, "upload of rho_init failed: %s", hipGetErrorString(e)));
        rho_st = st;
    }
    if (p->v_init) {
        if ((e = hipMemcpyAsync(st + N, p->v_init, (size_t)D * NB, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
            return cleanup(fail(LBM_ERR_HIP, "upload of v_init failed: %s", hipGetErrorString(e)));
        v_st = st + N;
    }
    // boundary-node list: cell, type | normal << 8, (v_b, rho_b) in the value type
    std::vector<uint32_t> bcell, bcode;
    std::vector<char> bval;
    if (nb) {
        bcell.reserve(nb);
        bcode.reserve(nb);
        bval.resize((size_t)nb * 4 * s);
        uint32_t k = 0;
        for (int64_t n = 0; n < N; ++n) {
            if (!p->bc_type[n]) continue;
            bcell.push_back((uint32_t)n);
            int o[3];
            decode_normal(p->bc_normal[n], D, o);
            bcode.push_back((uint32_t)p->bc_type[n] | (canonical_normal(o) << 8));
            double v4[4] = {0.0, 0.0, 0.0, p->bc_density ? p->bc_density[n] : p->rho0};
            if (p->bc_velocity)
                for (int a = 0; a < D; ++a) v4[a] = p->bc_velocity[(int64_t)a * N + n];
            for (int j = 0; j < 4; ++j) {
                if (s == 8) std::memcpy(bval.data() + ((size_t)k * 4 + j) * 8, &v4[j], 8);
                else {
                    const float x = (float)v4[j];
                    std::memcpy(bval.data() + ((size_t)k * 4 + j) * 4, &x, 4);
                }
            }
            ++k;
        }
        if ((e = hipMemcpyAsync(h->ws + L.bcell, bcell.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(h->ws + L.bcode, bcode.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(h->ws + L.bval, bval.data(), bval.size(), hipMemcpyHostToDevice, h->stream)) != hipSuccess)
            return cleanup(fail(LBM_ERR_HIP, "upload of boundary nodes failed: %s", hipGetErrorString(e)));
    }
    // analytic porosity derivatives, converted to the value type on the host (solid cells: 0)
    std::vector<char> dbuf;
    if (h->analytic) {
        const int K = D + D * (D + 1) / 2;
        dbuf.resize((size_t)K * N * s);
        for (int j = 0; j < K; ++j) {
            const double *src = j < D ? p->grad_eps + (int64_t)j * N : p->hess_eps + (int64_t)(j - D) * N;
            for (int64_t n = 0; n < N; ++n) {
                const double v = (p->mask && p->mask[n]) ? 0.0 : src[n];
                char *dst = dbuf.data() + ((size_t)j * N + n) * s;
                if (s == 8) std::memcpy(dst, &v, 8);
                else {
                    const float x = (float)v;
                    std::memcpy(dst, &x, 4);
                }
            }
        }
        if ((e = hipMemcpyAsync(h->ws + L.deps, dbuf.data(), dbuf.size(), hipMemcpyHostToDevice, h->stream)) != hipSuccess)
            return cleanup(fail(LBM_ERR_HIP, "upload of porosity derivatives failed: %s", hipGetErrorString(e)));
    }
    const uint8_t *mk = mask_ptr(h);
    const bool lag = p->scheme == LBM_SCHEME_LAGGED;
    if (h->storage == LBM_F64) {
        if (D == 2) hipLaunchKernelGGL((lbm::k_fill_init<2, double>), flat_grid(N), dim3(256), 0, h->stream, rho_st, v_st, mk, ws_ptr<lbm::P4<double>>(h, L.m2[0]), lag ? ws_ptr<lbm::P4<double>>(h, L.m1[0]) : nullptr, N, p->rho0);
        else hipLaunchKernelGGL((lbm::k_fill_init<3, double>), flat_grid(N), dim3(256), 0, h->stream, rho_st, v_st, mk, ws_ptr<lbm::P4<double>>(h, L.m2[0]), lag ? ws_ptr<lbm::P4<double>>(h, L.m1[0]) : nullptr, N, p->rho0);
    } else {
        if (D == 2) hipLaunchKernelGGL((lbm::k_fill_init<2, float>), flat_grid(N), dim3(256), 0, h->stream, rho_st, v_st, mk, ws_ptr<lbm::P4<float>>(h, L.m2[0]), lag ? ws_ptr<lbm::P4<float>>(h, L.m1[0]) : nullptr, N, p->rho0);
        else hipLaunchKernelGGL((lbm::k_fill_init<3, float>), flat_grid(N), dim3(256), 0, h->stream, rho_st, v_st, mk, ws_ptr<lbm::P4<float>>(h, L.m2[0]), lag ? ws_ptr<lbm::P4<float>>(h, L.m1[0]) : nullptr, N, p->rho0);
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return cleanup(fail(LBM_ERR_HIP, "initial-field kernel failed: %s", hipGetErrorString(e)));
    dispatch(h, InitPass{h});
    if ((e = hipGetLastError()) != hipSuccess)
        return cleanup(fail(LBM_ERR_HIP, "initial-population kernel failed: %s", hipGetErrorString(e)));
    // residual snapshot starts at zero
    if ((e = hipMemsetAsync(h->ws + L.vsnap, 0, (size_t)D * N * s, h->stream)) != hipSuccess)
        return cleanup(fail(LBM_ERR_HIP, "snapshot clear failed: %s", hipGetErrorString(e)));
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess)
        return cleanup(fail(LBM_ERR_HIP, "initialisation failed: %s", hipGetErrorString(e)));
    if (solids) {
        // share of solid-aware tiles, which decides the occupancy request of the kernels
        std::vector<uint8_t> flags(8 * (size_t)h->tiles.per);
        if ((e = hipMemcpyAsync(flags.data(), h->ws + L.tsolid, flags.size(),
                                hipMemcpyDeviceToHost, h->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(h->stream)) != hipSuccess)
            return cleanup(fail(LBM_ERR_HIP, "tile-flag read failed: %s", hipGetErrorString(e)));
        size_t aware = 0;
        for (uint8_t v : flags) aware += v != 0;
        h->solid_occ = 4 * aware < flags.size();
    }
    *out = h;
    return LBM_OK;
}

LBM_API int lbm_step(lbm_solver *h, int64_t n) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (n < 0) return fail(LBM_ERR_INVALID_ARG, "negative step count");
    for (int64_t k = 0; k < n; ++k) {
        hipError_t e = one_step(h, nullptr);
        if (e != hipSuccess) return fail(LBM_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    }
    return LBM_OK;
}

LBM_API int lbm_step_timed(lbm_solver *h, int64_t n, double kernel_ms[3]) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (n < 0 || !kernel_ms) return fail(LBM_ERR_INVALID_ARG, "bad step count or output");
    // Events bracket every kernel of a chunk of steps; the host waits once per chunk.
    constexpr int64_t kChunk = 2048;
    const int64_t nev = 3 * std::min<int64_t>(n, kChunk) + 1;
    std::vector<hipEvent_t> ev((size_t)nev);
    for (auto &x : ev) HIP_TRY(hipEventCreate(&x));
    double acc[3] = {0, 0, 0};
    int out = LBM_OK;
    for (int64_t done = 0; done < n && out == LBM_OK;) {
        const int64_t m = std::min<int64_t>(n - done, kChunk);
        hipError_t e = hipEventRecord(ev[0], h->stream);
        for (int64_t k = 0; k < m && e == hipSuccess; ++k) e = one_step(h, &ev[3 * k + 1]);
        if (e == hipSuccess) e = hipEventSynchronize(ev[3 * m]);
        if (e != hipSuccess) {
            out = fail(LBM_ERR_HIP, "timed step failed: %s", hipGetErrorString(e));
            break;
        }
        for (int64_t k = 0; k < m; ++k)
            for (int j = 0; j < 3; ++j) {
                // a two-pass step with the correction inside the collision pass has no
                // correction kernel: its share is 0 and the collision's interval spans both
                if (h->fused_vc && h->scheme == LBM_SCHEME_TWO_PASS && j == 1) continue;
                const int j0 = h->fused_vc && h->scheme == LBM_SCHEME_TWO_PASS && j == 2 ? 1 : j;
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, ev[3 * k + j0], ev[3 * k + j + 1]);
                acc[j] += ms;
            }
        done += m;
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    for (int j = 0; j < 3; ++j) kernel_ms[j] = acc[j];
    return out;
}

LBM_API int lbm_moments(lbm_solver *h, void *rho_dev, void *v_dev, int dtype, int velocity_kind) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_ERR_INVALID_ARG, "bad dtype");
    if (velocity_kind != LBM_VELOCITY_SUPERFICIAL && velocity_kind != LBM_VELOCITY_INTRINSIC)
        return fail(LBM_ERR_INVALID_ARG, "bad velocity_kind");
    const size_t m2 = current_moments(h);
    LAUNCH_CHECK();
    const int64_t N = h->N;
#define LBM_OUT(DD, TT, OO)                                                                      \
    hipLaunchKernelGGL((lbm::k_moments_out<DD, TT, OO>), flat_grid(N), dim3(256), 0, h->stream, \
                       ws_ptr<const lbm::P4<TT>>(h, m2), ws_ptr<const TT>(h, h->L.eps),           \
                       (OO *)rho_dev, (OO *)v_dev, N, velocity_kind)
    if (h->D == 2) {
        if (h->storage == LBM_F64) { if (dtype == LBM_DTYPE_F64) LBM_OUT(2, double, double); else LBM_OUT(2, double, float); }
        else { if (dtype == LBM_DTYPE_F64) LBM_OUT(2, float, double); else LBM_OUT(2, float, float); }
    } else {
        if (h->storage == LBM_F64) { if (dtype == LBM_DTYPE_F64) LBM_OUT(3, double, double); else LBM_OUT(3, double, float); }
        else { if (dtype == LBM_DTYPE_F64) LBM_OUT(3, float, double); else LBM_OUT(3, float, float); }
    }
#undef LBM_OUT
    LAUNCH_CHECK();
    return LBM_OK;
}

LBM_API int lbm_residual(lbm_solver *h, lbm_stats *out) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    rc = enqueue_stats(h);
    if (rc) return rc;
    double r[lbm::kStatsSlots];
    HIP_TRY(hipMemcpyAsync(r, h->ws + h->L.res, sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    out->mass = r[0];
    out->momentum[0] = r[1];
    out->momentum[1] = r[2];
    out->momentum[2] = h->D == 3 ? r[3] : 0.0;
    out->vmax = r[4];
    out->dv2 = r[5];
    out->v2 = r[6];
    out->residual = r[6] > 0 ? std::sqrt(r[5] / r[6]) : INFINITY;
    out->nonfinite = (int64_t)r[7];
    out->step = h->step;
    if (out->nonfinite > 0) return fail(LBM_ERR_NONFINITE, "%lld fluid cells are not finite", (long long)out->nonfinite);
    return LBM_OK;
}

LBM_API int lbm_stats_noalloc(lbm_solver *h, double *stats_dev) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!stats_dev) return fail(LBM_ERR_INVALID_ARG, "stats_dev is NULL");
    const int nblocks = stats_blocks(h);
    if (nblocks > lbm::kStatsBlocks)  // a guard: the reduction never uses more blocks
        return fail(LBM_ERR_UNSUPPORTED, "%d statistics blocks exceed the scratch of %d",
                    nblocks, lbm::kStatsBlocks);
    double *part = nullptr;
    rc = scratch_of_device(h->device, &part);
    if (rc) return rc;
    return enqueue_stats(h, part, stats_dev);
}

LBM_API int lbm_get_populations(lbm_solver *h, void *dev_out, int dtype) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!dev_out) return fail(LBM_ERR_INVALID_ARG, "dev_out is NULL");
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_ERR_INVALID_ARG, "bad dtype");
    // the unknown incoming populations of outflow nodes are those the next step uses
    if (h->bc_outflow) dispatch(h, BcOutflowPass{h});
    dispatch(h, ExportPass{h, dev_out, dtype});
    LAUNCH_CHECK();
    return LBM_OK;
}

LBM_API int lbm_set_populations(lbm_solver *h, const void *dev_in, int dtype, int64_t step) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!dev_in) return fail(LBM_ERR_INVALID_ARG, "dev_in is NULL");
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_ERR_INVALID_ARG, "bad dtype");
    if (step < 0) return fail(LBM_ERR_INVALID_ARG, "negative step");
    h->phase = 0;  // the import writes the natural layout
    dispatch(h, ImportPass{h, dev_in, dtype});
    LAUNCH_CHECK();
    h->phase = 0;
    h->step = step;
    h->have_prev = false;  // the lagged scheme's history restarts with a two-pass step
    return LBM_OK;
}

LBM_API int lbm_get_step(const lbm_solver *h, int64_t *step) {
    int rc = check_handle(h);
    if (rc) return rc;
    if (!step) return fail(LBM_ERR_INVALID_ARG, "step is NULL");
    *step = h->step;
    return LBM_OK;
}

LBM_API int lbm_destroy(lbm_solver *h) {
    delete h;
    return LBM_OK;
}

}  // extern "C"
