// lbm_server.hip -- request server of include/lbm.h: admission by workspace footprint into the
// caller's device pool, batched passes over all active runs, per-round statistics, retirement.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

// ------------------------------------------------------------------------------------------
// Batched passes.  One launch covers the tiles of every run of a group (same lattice, types,
// solids flag, scheme and AA phase).  Run r owns workgroups [starts[r], starts[r + 1]); each
// run's count is a multiple of 8, so workgroup w - starts[r] lands on the XCD the run's own
// tile order expects.  The run descriptor is uniform per workgroup and read through the
// scalar cache.
// ------------------------------------------------------------------------------------------
template <typename T, typename P>
struct RunDesc {
    P *f;
    const T *eps, *muD, *muF;
    const uint8_t *mask;
    P4<T> *m1[2];
    P4<T> *m2[2];
    Grid g;
    Tiling tl;
    Phys<T> ph;
    int cur;  // record pair holding the previous step's moments at the start of the round
};

__device__ __forceinline__ int find_run(const uint32_t *__restrict__ starts, int nrun,
                                        uint32_t w) {
    int lo = 0, hi = nrun - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int D, typename T, typename P, bool S, int PH>
__global__ __launch_bounds__(256) void kb_moments(const RunDesc<T, P> *__restrict__ runs,
                                                  const uint32_t *__restrict__ starts, int nrun) {
    const int r = find_run(starts, nrun, blockIdx.x);
    const RunDesc<T, P> &d = runs[r];
    moments_body<D, T, P, S, PH, false>(d.f, d.eps, d.muD, d.muF, d.mask, d.m1[0], nullptr, d.g, d.tl,
                                 d.ph, blockIdx.x - starts[r]);
}

template <int D, typename T, typename P, bool S>
__global__ __launch_bounds__(256) void kb_vcorrect(const RunDesc<T, P> *__restrict__ runs,
                                                   const uint32_t *__restrict__ starts, int nrun) {
    const int r = find_run(starts, nrun, blockIdx.x);
    const RunDesc<T, P> &d = runs[r];
    vcorrect_body<D, T, S, false>(d.m1[0], d.m1[0], d.eps, d.mask, d.m2[0], d.g, d.tl, d.ph,
                           blockIdx.x - starts[r]);
}

template <int D, typename T, typename P, bool S, int PH>
__global__ __launch_bounds__(256) void kb_collide(const RunDesc<T, P> *__restrict__ runs,
                                                  const uint32_t *__restrict__ starts, int nrun) {
    const int r = find_run(starts, nrun, blockIdx.x);
    const RunDesc<T, P> &d = runs[r];
    collide_body<D, T, P, S, PH, false>(d.f, d.m2[0], d.m2[0], d.eps, d.muD, d.muF, d.mask, d.g,
                                        d.tl, d.ph, blockIdx.x - starts[r]);
}

// parity: the step's position in the round (mod 2); the previous records alternate with it.
template <int D, typename T, typename P, bool S, int PH>
__global__ __launch_bounds__(256) void kb_fused(const RunDesc<T, P> *__restrict__ runs,
                                                const uint32_t *__restrict__ starts, int nrun,
                                                int parity) {
    const int r = find_run(starts, nrun, blockIdx.x);
    const RunDesc<T, P> &d = runs[r];
    const int prev = d.cur ^ parity;
    fused_body<D, T, P, S, PH, false>(d.f, d.m1[prev], d.m2[prev], d.m1[prev ^ 1], d.m2[prev ^ 1],
                               d.eps, d.muD, d.muF, d.mask, d.g, d.tl, d.ph,
                               blockIdx.x - starts[r]);
}

}  // namespace lbm

namespace lbmh {

// First-fit allocator over the device pool, in 256-byte granules; adjacent free ranges merge.
class PoolAllocator {
public:
    void init(size_t base, size_t size) {
        free_.clear();
        if (size) free_[base] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (const auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

private:
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    int state = LBM_REQ_QUEUED;
    lbm_params p{};
    std::vector<double> eps, kappa, forch, rho_init, v_init;
    std::vector<double> bc_velocity, bc_density, grad_eps, hess_eps;
    std::vector<uint8_t> mask, bc_type, bc_normal;
    // stepped on its own (lbm_step) instead of in the batched launches: wet-node boundaries,
    // Picard iterations or analytic porosity derivatives
    bool solo = false;
    double tol = 0;
    int64_t max_steps = 0;
    int floor_checks = 0;       // rounds without a new minimum of the residual before retiring
    double best = INFINITY;     // lowest residual so far (new minima count when 1 % lower)
    int since_best = 0;         // rounds since the last new minimum
    size_t bytes = 0, off = 0;
    bool holds_memory = false;
    lbm_solver *h = nullptr;
    double residual = INFINITY;
    int64_t steps = 0;
    double t_submit = 0, t_admit = -1, t_done = -1;
    int64_t cells = 0;
    int waited = 0;  // rounds spent queued behind backfilled requests
};

constexpr int kMaxRuns = 4096;
constexpr int kStarvationRounds = 64;
// descriptor table: the largest descriptor per run plus one start index per run and group
constexpr size_t kTableBytes =
    (size_t)kMaxRuns * (sizeof(lbm::RunDesc<double, double>) + 2 * sizeof(uint32_t)) + 64 * 1024;

}  // namespace lbmh

struct lbm_server {
    char *pool = nullptr;
    size_t pool_bytes = 0;
    hipStream_t stream = nullptr;
    int64_t check_every = 100;
    int max_active = 0;
    lbmh::PoolAllocator alloc;
    size_t table_off = 0;
    std::vector<std::unique_ptr<lbmh::Request>> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> active;
    double *pinned = nullptr;  // kMaxRuns x kStatsSlots statistics, host side
    std::vector<char> table_host;
    std::chrono::steady_clock::time_point t0;
    int64_t rounds = 0, admitted = 0, finished = 0;
    double cell_updates = 0;
    size_t pool_used = 0, pool_peak = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace lbmh {
namespace {

// One group of runs launched together.
struct Group {
    int D, storage, scheme;
    bool solids;
    std::vector<lbmh::Request *> runs;
    size_t desc_off = 0, starts_off = 0;  // device offsets in the pool
    uint32_t nwg = 0;
};

template <int D, typename T, typename P, bool S>
struct GroupOps {
    using Desc = lbm::RunDesc<T, P>;

    // Append the group's descriptors and start indices to the host table.
    static void fill(lbm_server *sv, Group &gr, std::vector<char> &tab) {
        size_t at = align256(tab.size());
        gr.desc_off = sv->table_off + at;
        tab.resize(at + gr.runs.size() * sizeof(Desc));
        uint32_t wg = 0;
        std::vector<uint32_t> starts;
        for (size_t k = 0; k < gr.runs.size(); ++k) {
            const lbm_solver *h = gr.runs[k]->h;
            Desc d;
            d.f = ws_ptr<P>(h, h->L.f);
            d.eps = ws_ptr<const T>(h, h->L.eps);
            d.muD = ws_ptr<const T>(h, h->L.muD);
            d.muF = ws_ptr<const T>(h, h->L.muF);
            d.mask = mask_ptr(h);
            for (int j = 0; j < 2; ++j) {
                d.m1[j] = ws_ptr<lbm::P4<T>>(h, h->L.m1[j]);
                d.m2[j] = ws_ptr<lbm::P4<T>>(h, h->L.m2[j]);
            }
            d.g = grid_of(h);
            d.tl = h->tiles;
            d.ph = phys_of<T>(h);
            d.cur = h->cur;
            std::memcpy(tab.data() + at + k * sizeof(Desc), &d, sizeof(Desc));
            starts.push_back(wg);
            wg += 8u * h->tiles.per;
        }
        gr.nwg = wg;
        at = align256(tab.size());
        gr.starts_off = sv->table_off + at;
        tab.resize(at + starts.size() * sizeof(uint32_t));
        std::memcpy(tab.data() + at, starts.data(), starts.size() * sizeof(uint32_t));
    }

    template <int PH>
    static void step_ph(lbm_server *sv, const Group &gr, int parity) {
        const Desc *runs = reinterpret_cast<const Desc *>(sv->pool + gr.desc_off);
        const uint32_t *starts = reinterpret_cast<const uint32_t *>(sv->pool + gr.starts_off);
        const int n = (int)gr.runs.size();
        if (gr.scheme == LBM_SCHEME_LAGGED) {
            hipLaunchKernelGGL((lbm::kb_fused<D, T, P, S, PH>), dim3(gr.nwg), dim3(256), 0,
                               sv->stream, runs, starts, n, parity);
        } else {
            hipLaunchKernelGGL((lbm::kb_moments<D, T, P, S, PH>), dim3(gr.nwg), dim3(256), 0,
                               sv->stream, runs, starts, n);
            hipLaunchKernelGGL((lbm::kb_vcorrect<D, T, P, S>), dim3(gr.nwg), dim3(256), 0,
                               sv->stream, runs, starts, n);
            hipLaunchKernelGGL((lbm::kb_collide<D, T, P, S, PH>), dim3(gr.nwg), dim3(256), 0,
                               sv->stream, runs, starts, n);
        }
    }

    // Step k of the round: every run starts the round in the natural layout (phase 0).
    static void step(lbm_server *sv, const Group &gr, int64_t k) {
        if (k & 1) step_ph<1>(sv, gr, 1);
        else step_ph<0>(sv, gr, 0);
    }
};

template <typename F>
void group_dispatch(const Group &gr, F &&fn) {
#define LBM_G(DD, TT, PP)                                        \
    if (gr.solids) fn.template operator()<DD, TT, PP, true>();   \
    else fn.template operator()<DD, TT, PP, false>();
#define LBM_GD(DD)                                                       \
    switch (gr.storage) {                                                \
    case LBM_F64: { LBM_G(DD, double, double) } break;                   \
    case LBM_F32: { LBM_G(DD, float, float) } break;                     \
    case LBM_F16_SHIFTED: { LBM_G(DD, float, _Float16) } break;          \
    default: { LBM_G(DD, float, __bf16) } break;                         \
    }
    if (gr.D == 2) { LBM_GD(2) }
    else { LBM_GD(3) }
#undef LBM_GD
#undef LBM_G
}

struct FillOp {
    lbm_server *sv;
    Group &gr;
    std::vector<char> &tab;
    template <int D, typename T, typename P, bool S>
    void operator()() { GroupOps<D, T, P, S>::fill(sv, gr, tab); }
};
struct StepOp {
    lbm_server *sv;
    const Group &gr;
    int64_t k;
    template <int D, typename T, typename P, bool S>
    void operator()() { GroupOps<D, T, P, S>::step(sv, gr, k); }
};

int check_server(const lbm_server *s) {
    if (!s) return fail(LBM_ERR_INVALID_ARG, "null server handle");
    return LBM_OK;
}

lbmh::Request *find_req(const lbm_server *s, int64_t id) {
    if (id < 0 || id >= (int64_t)s->reqs.size()) return nullptr;
    return s->reqs[(size_t)id].get();
}

void free_run(lbm_server *s, lbmh::Request *q) {
    if (q->h) {
        lbm_destroy(q->h);
        q->h = nullptr;
    }
    if (q->holds_memory) {
        s->alloc.release(q->off, q->bytes);
        s->pool_used -= align256(q->bytes);
        q->holds_memory = false;
    }
}

// Admit queued requests in arrival order; later ones may pass a request that does not fit
// until it has waited kStarvationRounds rounds.
int admit(lbm_server *s) {
    std::deque<int64_t> keep;
    bool blocked = false;
    while (!s->queue.empty()) {
        const int64_t id = s->queue.front();
        s->queue.pop_front();
        lbmh::Request *q = find_req(s, id);
        const bool room = (s->max_active == 0 || (int)s->active.size() < s->max_active) &&
                          (int)s->active.size() < kMaxRuns;
        size_t off = 0;
        if (blocked || !room || !s->alloc.alloc(q->bytes, &off)) {
            if (!blocked && room) {
                q->waited += 1;
                if (q->waited >= kStarvationRounds) blocked = true;
            }
            keep.push_back(id);
            continue;
        }
        q->off = off;
        q->holds_memory = true;
        s->pool_used += align256(q->bytes);
        s->pool_peak = std::max(s->pool_peak, s->pool_used);
        const int rc = lbm_create(&q->p, s->pool + off, q->bytes, s->stream, &q->h);
        if (rc != LBM_OK) {
            q->state = LBM_REQ_FAILED;
            q->t_done = s->now();
            free_run(s, q);
            s->finished += 1;
            continue;
        }
        q->state = LBM_REQ_ACTIVE;
        q->t_admit = s->now();
        s->active.push_back(id);
        s->admitted += 1;
        // the first statistics call only takes the velocity snapshot
        if (lbmh::enqueue_stats(q->h) != LBM_OK) return LBM_ERR_HIP;
    }
    s->queue.swap(keep);
    return LBM_OK;
}

}  // namespace
}  // namespace lbmh

using namespace lbmh;

extern "C" {

LBM_API int lbm_server_create(void *dev_pool, size_t pool_bytes, int64_t check_every,
                              int max_active, void *hip_stream, lbm_server **out) {
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!dev_pool) return fail(LBM_ERR_INVALID_ARG, "dev_pool is NULL");
    if (reinterpret_cast<uintptr_t>(dev_pool) % 256)
        return fail(LBM_ERR_WORKSPACE, "dev_pool must be 256-byte aligned");
    if (pool_bytes < (size_t(1) << 20) || pool_bytes < 2 * kTableBytes)
        return fail(LBM_ERR_WORKSPACE, "a pool of %zu bytes is too small", pool_bytes);
    if (check_every < 2 || (check_every & 1))
        return fail(LBM_ERR_INVALID_ARG, "check_every must be even and >= 2");
    if (max_active < 0) return fail(LBM_ERR_INVALID_ARG, "max_active must be >= 0");
    lbm_server *s = new (std::nothrow) lbm_server();
    if (!s) return fail(LBM_ERR_INVALID_ARG, "out of host memory");
    s->pool = reinterpret_cast<char *>(dev_pool);
    s->pool_bytes = pool_bytes;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->check_every = check_every;
    s->max_active = max_active;
    s->table_off = 0;
    s->alloc.init(align256(kTableBytes), pool_bytes - align256(kTableBytes));
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return LBM_OK;
}

LBM_API int lbm_server_submit(lbm_server *s, const lbm_params *p, double tol, int64_t max_steps,
                              int floor_checks, int64_t *id) {
    int rc = check_server(s);
    if (rc) return rc;
    if (!p || !id) return fail(LBM_ERR_INVALID_ARG, "null argument");
    if (!(tol > 0) || max_steps < s->check_every)
        return fail(LBM_ERR_INVALID_ARG, "tol must be > 0 and max_steps >= check_every");
    if (floor_checks < 0) return fail(LBM_ERR_INVALID_ARG, "floor_checks must be >= 0");
    size_t bytes = 0;
    rc = lbm_footprint(p, &bytes);
    if (rc) return rc;
    if (align256(bytes) > s->pool_bytes - align256(kTableBytes))
        return fail(LBM_ERR_WORKSPACE, "a workspace of %zu bytes can never fit the pool", bytes);
    if (!p->eps || !p->kappa || !p->forch) return fail(LBM_ERR_INVALID_ARG, "eps, kappa and forch are required");
    auto q = std::unique_ptr<Request>(new (std::nothrow) Request());
    if (!q) return fail(LBM_ERR_INVALID_ARG, "out of host memory");
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const int D = p->lattice == LBM_D2Q9 ? 2 : 3;
    q->p = *p;
    q->eps.assign(p->eps, p->eps + N);
    q->kappa.assign(p->kappa, p->kappa + N);
    q->forch.assign(p->forch, p->forch + N);
    q->p.eps = q->eps.data();
    q->p.kappa = q->kappa.data();
    q->p.forch = q->forch.data();
    if (p->mask) {
        q->mask.assign(p->mask, p->mask + N);
        q->p.mask = q->mask.data();
    }
    if (p->rho_init) {
        q->rho_init.assign(p->rho_init, p->rho_init + N);
        q->p.rho_init = q->rho_init.data();
    }
    if (p->v_init) {
        q->v_init.assign(p->v_init, p->v_init + (size_t)D * N);
        q->p.v_init = q->v_init.data();
    }
    if (p->bc_type) {
        q->bc_type.assign(p->bc_type, p->bc_type + N);
        q->p.bc_type = q->bc_type.data();
    }
    if (p->bc_type && p->bc_normal) {
        q->bc_normal.assign(p->bc_normal, p->bc_normal + N);
        q->p.bc_normal = q->bc_normal.data();
    }
    if (p->bc_type && p->bc_velocity) {
        q->bc_velocity.assign(p->bc_velocity, p->bc_velocity + (size_t)D * N);
        q->p.bc_velocity = q->bc_velocity.data();
    }
    if (p->bc_type && p->bc_density) {
        q->bc_density.assign(p->bc_density, p->bc_density + N);
        q->p.bc_density = q->bc_density.data();
    }
    if (p->grad_eps) {
        q->grad_eps.assign(p->grad_eps, p->grad_eps + (size_t)D * N);
        q->p.grad_eps = q->grad_eps.data();
    }
    if (p->hess_eps) {
        q->hess_eps.assign(p->hess_eps, p->hess_eps + (size_t)(D * (D + 1) / 2) * N);
        q->p.hess_eps = q->hess_eps.data();
    }
    q->solo = p->bc_type || p->picard_iters || p->grad_eps || p->hess_eps;
    q->id = (int64_t)s->reqs.size();
    q->tol = tol;
    q->max_steps = max_steps;
    q->floor_checks = floor_checks;
    q->bytes = bytes;
    q->cells = (int64_t)N;
    q->t_submit = s->now();
    *id = q->id;
    s->queue.push_back(q->id);
    s->reqs.push_back(std::move(q));
    return LBM_OK;
}

LBM_API int lbm_server_progress(lbm_server *s, int64_t max_rounds, int64_t *finished_ids,
                                int max_finished, int *n_finished) {
    int rc = check_server(s);
    if (rc) return rc;
    if (max_rounds < 0 || (max_finished > 0 && !finished_ids))
        return fail(LBM_ERR_INVALID_ARG, "bad arguments");
    if (!s->pinned) {  // first device work: pinned host buffer for the per-round statistics
        HIP_TRY(hipHostMalloc((void **)&s->pinned, sizeof(double) * kMaxRuns * lbm::kStatsSlots,
                              hipHostMallocDefault));
    }
    int nf = 0;
    for (int64_t round = 0; round < max_rounds; ++round) {
        rc = admit(s);
        if (rc) return fail(rc, "admission failed");
        if (s->active.empty()) break;
        // groups of runs that share kernels; runs with per-run boundary kernels or iterations
        // step on their own
        std::vector<Group> groups;
        std::vector<Request *> solo;
        for (int64_t id : s->active) {
            Request *q = find_req(s, id);
            if (q->solo) {
                solo.push_back(q);
                continue;
            }
            const lbm_solver *h = q->h;
            const bool solids = h->solids;
            Group *g = nullptr;
            for (auto &x : groups)
                if (x.D == h->D && x.storage == h->storage && x.scheme == h->scheme &&
                    x.solids == solids)
                    g = &x;
            if (!g) {
                groups.push_back(Group{h->D, h->storage, h->scheme, solids, {}});
                g = &groups.back();
            }
            g->runs.push_back(q);
        }
        s->table_host.clear();
        for (auto &g : groups) group_dispatch(g, FillOp{s, g, s->table_host});
        HIP_TRY(hipMemcpyAsync(s->pool + s->table_off, s->table_host.data(), s->table_host.size(),
                               hipMemcpyHostToDevice, s->stream));
        for (int64_t k = 0; k < s->check_every; ++k)
            for (const auto &g : groups) group_dispatch(g, StepOp{s, g, k});
        LAUNCH_CHECK();
        for (Request *q : solo) {  // advances the run's own step count, phase and records
            rc = lbm_step(q->h, s->check_every);
            if (rc) return rc;
        }
        // statistics of every run, one synchronisation
        for (size_t r = 0; r < s->active.size(); ++r) {
            Request *q = find_req(s, s->active[r]);
            lbm_solver *h = q->h;
            if (!q->solo)  // the round length is even: phase and records unchanged
                h->step += s->check_every;
            q->steps = h->step;
            s->cell_updates += (double)q->cells * (double)s->check_every;
            if (enqueue_stats(h) != LBM_OK) return LBM_ERR_HIP;
            HIP_TRY(hipMemcpyAsync(s->pinned + r * lbm::kStatsSlots, h->ws + h->L.res,
                                   sizeof(double) * lbm::kStatsSlots, hipMemcpyDeviceToHost,
                                   s->stream));
        }
        HIP_TRY(hipStreamSynchronize(s->stream));
        s->rounds += 1;
        const double t = s->now();
        std::vector<int64_t> still;
        for (size_t r = 0; r < s->active.size(); ++r) {
            Request *q = find_req(s, s->active[r]);
            const double *st = s->pinned + r * lbm::kStatsSlots;
            q->residual = st[6] > 0 ? std::sqrt(st[5] / st[6]) : INFINITY;
            // a new minimum counts when it is at least 1 % below the previous one, so that the
            // slow drift of the lowest value of a residual that fluctuates about its floor
            // does not
            if (q->residual < 0.99 * q->best) {
                q->best = q->residual;
                q->since_best = 0;
            } else {
                q->since_best += 1;
            }
            int state = LBM_REQ_ACTIVE;
            if (st[7] > 0) state = LBM_REQ_FAILED;
            else if (q->residual < q->tol) state = LBM_REQ_CONVERGED;
            else if (q->floor_checks > 0 && q->since_best >= q->floor_checks)
                state = LBM_REQ_FLOOR;
            else if (q->h->step >= q->max_steps) state = LBM_REQ_CENSORED;
            if (state == LBM_REQ_ACTIVE) {
                still.push_back(q->id);
                continue;
            }
            q->state = state;
            q->t_done = t;
            s->finished += 1;
            if (nf < max_finished) finished_ids[nf] = q->id;
            nf += 1;
        }
        s->active.swap(still);
    }
    if (n_finished) *n_finished = nf;
    return LBM_OK;
}

LBM_API int lbm_server_info(const lbm_server *s, int64_t id, lbm_request_info *out) {
    int rc = check_server(s);
    if (rc) return rc;
    const Request *q = find_req(s, id);
    if (!q || !out) return fail(LBM_ERR_INVALID_ARG, "unknown request %lld or null output", (long long)id);
    out->id = q->id;
    out->state = q->state;
    out->steps = q->steps;
    out->residual = q->residual;
    out->t_submit = q->t_submit;
    out->t_admit = q->t_admit;
    out->t_done = q->t_done;
    out->cells = q->cells;
    out->workspace_bytes = q->bytes;
    return LBM_OK;
}

LBM_API int lbm_server_solver(lbm_server *s, int64_t id, lbm_solver **out) {
    int rc = check_server(s);
    if (rc) return rc;
    Request *q = find_req(s, id);
    if (!q || !out) return fail(LBM_ERR_INVALID_ARG, "unknown request %lld or null output", (long long)id);
    if (!q->h) return fail(LBM_ERR_STATE, "request %lld holds no state (queued, failed or released)", (long long)id);
    *out = q->h;
    return LBM_OK;
}

LBM_API int lbm_server_release(lbm_server *s, int64_t id) {
    int rc = check_server(s);
    if (rc) return rc;
    Request *q = find_req(s, id);
    if (!q) return fail(LBM_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    if (q->state == LBM_REQ_QUEUED || q->state == LBM_REQ_ACTIVE)
        return fail(LBM_ERR_STATE, "request %lld has not finished", (long long)id);
    if (q->holds_memory) {
        // the last round's work on this run has completed (progress synchronised); later calls
        // through lbm_server_solver may still be queued on the stream
        HIP_TRY(hipStreamSynchronize(s->stream));
        free_run(s, q);
    }
    return LBM_OK;
}

LBM_API int lbm_server_get_stats(const lbm_server *s, lbm_server_stats *out) {
    int rc = check_server(s);
    if (rc) return rc;
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    out->rounds = s->rounds;
    out->submitted = (int64_t)s->reqs.size();
    out->admitted = s->admitted;
    out->finished = s->finished;
    out->queued = (int64_t)s->queue.size();
    out->active = (int64_t)s->active.size();
    out->cell_updates = s->cell_updates;
    out->pool_bytes = s->pool_bytes;
    out->pool_used = s->pool_used;
    out->pool_peak = s->pool_peak;
    return LBM_OK;
}

LBM_API int lbm_server_destroy(lbm_server *s) {
    if (!s) return LBM_OK;
    if (s->pinned) {  // device work was enqueued
        (void)hipStreamSynchronize(s->stream);
        for (auto &q : s->reqs) free_run(s, q.get());
        (void)hipHostFree(s->pinned);
    }
    delete s;
    return LBM_OK;
}

}  // extern "C"
