// ns_batch.hip -- many independent solves advanced together.
//
// A host-side scheduler: every member keeps its own fused launch plan
// (grid, physics, launch shape, workspace carve-up) and a batch step
// enqueues one RK3 step of each member that still has steps left.  Members
// are spread over a few internal streams (balanced by grid points), so the
// small grids' launches overlap on the device; the internal streams fork
// from and join back into the caller's stream, so the batch is ordered like
// any other stream work.  The launches are exactly rk3_step's, so a
// member's result does not depend on which other members share the batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

constexpr int kMaxStreams = 8;
constexpr int kMaxInstances = 4096;

struct Member {
    bool used = false;
    FusedPlan plan;
    double dt = 0.0;
    int steps_left = -1, steps_done = 0;
    int stream = 0;
    int64_t points = 0;
    const char *state_lo = nullptr, *state_hi = nullptr;
    const char *work_lo = nullptr, *work_hi = nullptr;
};

struct Batch {
    int max_inst = 0, nstreams = 0;
    ns_precision prec = NS_FP64;
    bool diag = false;
    ns_diag *d_diag = nullptr;
    hipStream_t streams[kMaxStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMaxStreams] = {};
    int64_t load[kMaxStreams] = {};
    std::vector<Member> m;
};

static void destroy(Batch *b)
{
    for (int i = 0; i < kMaxStreams; ++i) {
        if (b->streams[i]) {
            (void)hipStreamSynchronize(b->streams[i]);
            (void)hipStreamDestroy(b->streams[i]);
        }
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->d_diag) (void)hipFree(b->d_diag);
}

static bool overlaps(const char *a0, const char *a1, const char *b0, const char *b1)
{
    return a0 < b1 && b0 < a1;
}

}  // namespace ns

using namespace ns;

struct ns_batch : Batch {};

extern "C" {

ns_status ns_batch_create(int32_t max_instances, ns_precision prec, int32_t nstreams,
                          int32_t with_diagnostics, ns_batch **out)
{
    if (!out) return NS_ERR_ARG;
    *out = nullptr;
    if (max_instances < 1 || max_instances > kMaxInstances) return NS_ERR_ARG;
    if (prec != NS_FP64 && prec != NS_FP32_STORE) return NS_ERR_ARG;
    if (nstreams < 1 || nstreams > kMaxStreams) return NS_ERR_ARG;
    ns_batch *b = new (std::nothrow) ns_batch();
    if (!b) return NS_ERR_DEVICE;
    b->max_inst = max_instances;
    b->nstreams = nstreams;
    b->prec = prec;
    b->diag = with_diagnostics != 0;
    b->m.resize(max_instances);
    bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < nstreams; ++i) {
        // default priority; does not synchronise with the null stream
        ok = hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) == hipSuccess;
    }
    if (ok && b->diag) {
        const size_t bytes = (size_t)max_instances * sizeof(ns_diag);
        ok = hipMalloc((void **)&b->d_diag, bytes) == hipSuccess &&
             hipMemset(b->d_diag, 0, bytes) == hipSuccess;
    }
    if (!ok) {
        destroy(b);
        delete b;
        return NS_ERR_DEVICE;
    }
    *out = b;
    return NS_OK;
}

ns_status ns_batch_destroy(ns_batch *b)
{
    if (!b) return NS_ERR_ARG;
    destroy(b);
    delete b;
    return NS_OK;
}

ns_status ns_batch_add(ns_batch *b, const ns_instance *inst, int32_t *slot)
{
    if (!b || !inst || !slot) return NS_ERR_ARG;
    if (!std::isfinite(inst->dt) || !(inst->dt > 0.0) || inst->steps < 0) return NS_ERR_ARG;
    FusedPlan f;
    ns_status st = make_fused_plan(&inst->p, b->prec, inst->tile, inst->zchunk, inst->state,
                                   inst->work, inst->work_bytes, &f);
    if (st != NS_OK) return st;
    const char *s0 = (const char *)inst->state;
    const char *s1 = s0 + 5 * (size_t)f.c.N * sizeof(double);
    const char *w0 = (const char *)inst->work;
    const char *w1 = w0 + inst->work_bytes;
    if (overlaps(s0, s1, w0, w1)) return NS_ERR_ARG;
    int free_slot = -1;
    for (int i = 0; i < b->max_inst; ++i) {
        const Member &o = b->m[i];
        if (!o.used) {
            if (free_slot < 0) free_slot = i;
            continue;
        }
        // a member's buffers may not be shared with another member
        if (overlaps(s0, s1, o.state_lo, o.state_hi) || overlaps(s0, s1, o.work_lo, o.work_hi) ||
            overlaps(w0, w1, o.state_lo, o.state_hi) || overlaps(w0, w1, o.work_lo, o.work_hi))
            return NS_ERR_ARG;
    }
    if (free_slot < 0) return NS_ERR_WORKSPACE;
    int best = 0;
    for (int s = 1; s < b->nstreams; ++s)
        if (b->load[s] < b->load[best]) best = s;
    Member &m = b->m[free_slot];
    m.used = true;
    m.plan = f;
    m.dt = inst->dt;
    m.steps_left = inst->steps;
    m.steps_done = 0;
    m.stream = best;
    m.points = f.c.N;
    m.state_lo = s0;
    m.state_hi = s1;
    m.work_lo = w0;
    m.work_hi = w1;
    b->load[best] += m.points;
    *slot = free_slot;
    return NS_OK;
}

ns_status ns_batch_remove(ns_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_inst || !b->m[slot].used) return NS_ERR_ARG;
    Member &m = b->m[slot];
    b->load[m.stream] -= m.points;
    m = Member();
    return NS_OK;
}

ns_status ns_batch_step(ns_batch *b, int32_t nsteps, void *stream)
{
    if (!b || nsteps < 0) return NS_ERR_ARG;
    hipStream_t caller = (hipStream_t)stream;
    bool any = false;
    for (const Member &m : b->m) any = any || (m.used && m.steps_left > 0);
    if (!any || nsteps == 0) return NS_OK;
    NS_HIP_OK(hipEventRecord(b->fork, caller));
    for (int s = 0; s < b->nstreams; ++s) NS_HIP_OK(hipStreamWaitEvent(b->streams[s], b->fork, 0));
    // Largest members first within a step, so that small grids (which
    // cannot fill the device alone) run beside large ones on the other
    // streams.
    std::vector<int> order;
    for (int i = 0; i < b->max_inst; ++i)
        if (b->m[i].used) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->m[x].points > b->m[y].points; });
    // Step-major order: every member's step k is queued before any step
    // k + 1, so each internal stream is fed as the host walks the list.
    for (int32_t k = 0; k < nsteps; ++k) {
        for (int i : order) {
            Member &m = b->m[i];
            if (m.steps_left <= 0) continue;
            ns_diag *d = b->diag ? b->d_diag + i : nullptr;
            NS_HIP_OK(enqueue_fused_step(m.plan, m.dt, d, b->streams[m.stream]));
            --m.steps_left;
            ++m.steps_done;
        }
    }
    for (int s = 0; s < b->nstreams; ++s) {
        NS_HIP_OK(hipEventRecord(b->join[s], b->streams[s]));
        NS_HIP_OK(hipStreamWaitEvent(caller, b->join[s], 0));
    }
    return NS_OK;
}

ns_status ns_batch_poll(ns_batch *b, int32_t *steps_left, int32_t *steps_done, ns_diag *diag,
                        void *stream)
{
    if (!b) return NS_ERR_ARG;
    if (diag && !b->diag) return NS_ERR_ARG;
    for (int i = 0; i < b->max_inst; ++i) {
        const Member &m = b->m[i];
        if (steps_left) steps_left[i] = m.used ? m.steps_left : -1;
        if (steps_done) steps_done[i] = m.used ? m.steps_done : 0;
    }
    if (diag) {
        hipStream_t s = (hipStream_t)stream;
        NS_HIP_OK(hipMemcpyAsync(diag, b->d_diag, (size_t)b->max_inst * sizeof(ns_diag),
                                 hipMemcpyDeviceToHost, s));
        NS_HIP_OK(hipStreamSynchronize(s));
    }
    return NS_OK;
}

ns_status ns_batch_info(const ns_batch *b, int32_t *max_instances, int32_t *active,
                        int32_t *nstreams)
{
    if (!b) return NS_ERR_ARG;
    int a = 0;
    for (const Member &m : b->m) a += m.used ? 1 : 0;
    if (max_instances) *max_instances = b->max_inst;
    if (active) *active = a;
    if (nstreams) *nstreams = b->nstreams;
    return NS_OK;
}

}  // extern "C"
