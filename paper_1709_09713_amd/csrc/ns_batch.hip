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
//
// Optionally (ns_batch_set_graphs) kGraphSteps batch steps -- every
// stepping member's stage launches on their streams, forked from and joined
// into a batch-owned origin stream -- are captured once into a HIP graph
// and replayed while the set of stepping members stays the same (steps
// that do not fill a whole graph run eagerly); the graph is captured again
// when a member is added, removed or runs out of steps.  Every kernel
// argument is the same from step to step, so a replay is exactly the eager
// steps.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

constexpr int kMaxStreams = 8;
constexpr int32_t kGraphSteps = 8;   // steps per captured graph
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
    // graph replay
    bool graphs = false;
    hipStream_t origin = nullptr;       // capture and replay stream
    hipEvent_t gin = nullptr, gout = nullptr;
    hipGraphExec_t gexec = nullptr;     // one step of the current stepping set
};

static void drop_graph(Batch *b)
{
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
}

static void destroy(Batch *b)
{
    if (b->origin) (void)hipStreamSynchronize(b->origin);
    drop_graph(b);
    if (b->origin) (void)hipStreamDestroy(b->origin);
    if (b->gin) (void)hipEventDestroy(b->gin);
    if (b->gout) (void)hipEventDestroy(b->gout);
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

// Slots with steps left, largest grids first (stable), so that small grids,
// which cannot fill the device alone, run beside large ones on the other
// streams.
static std::vector<int> stepping_order(const Batch *b)
{
    std::vector<int> order;
    for (int i = 0; i < b->max_inst; ++i)
        if (b->m[i].used && b->m[i].steps_left > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->m[x].points > b->m[y].points; });
    return order;
}

// Queue nsteps steps of the members in `order`, forked once from `s` and
// joined once back into it.  Step-major: every member's step r is queued
// before step r + 1, so each internal stream is fed as the host walks the
// list and runs ahead of the others as far as its own work allows.
static hipError_t enqueue_steps(Batch *b, const std::vector<int> &order, int32_t nsteps, hipStream_t s)
{
    hipError_t e = hipEventRecord(b->fork, s);
    for (int k = 0; e == hipSuccess && k < b->nstreams; ++k) e = hipStreamWaitEvent(b->streams[k], b->fork, 0);
    for (int32_t r = 0; r < nsteps; ++r) {
        for (size_t j = 0; e == hipSuccess && j < order.size(); ++j) {
            const int i = order[j];
            const Member &m = b->m[i];
            ns_diag *d = b->diag ? b->d_diag + i : nullptr;
            e = enqueue_fused_step(m.plan, m.dt, d, b->streams[m.stream]);
        }
    }
    for (int k = 0; e == hipSuccess && k < b->nstreams; ++k) {
        e = hipEventRecord(b->join[k], b->streams[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[k], 0);
    }
    return e;
}

// Capture kGraphSteps steps of `order` on the origin stream into b->gexec.
static hipError_t capture_steps(Batch *b, const std::vector<int> &order)
{
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->origin, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    const hipError_t eq = enqueue_steps(b, order, kGraphSteps, b->origin);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->origin, &g);
    if (eq != hipSuccess) e = eq;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) b->gexec = nullptr;
    return e;
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
    if (!b) return NS_ERR_NOMEM;
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
    ns_status fail = NS_ERR_DEVICE;
    if (ok && b->diag) {
        const size_t bytes = (size_t)max_instances * sizeof(ns_diag);
        const hipError_t e = hipMalloc((void **)&b->d_diag, bytes);
        if (e == hipErrorOutOfMemory) fail = NS_ERR_NOMEM;
        ok = e == hipSuccess && hipMemset(b->d_diag, 0, bytes) == hipSuccess;
    }
    if (!ok) {
        destroy(b);
        delete b;
        return fail;
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
    drop_graph(b);
    return NS_OK;
}

ns_status ns_batch_remove(ns_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_inst || !b->m[slot].used) return NS_ERR_ARG;
    Member &m = b->m[slot];
    b->load[m.stream] -= m.points;
    m = Member();
    drop_graph(b);
    return NS_OK;
}

ns_status ns_batch_step(ns_batch *b, int32_t nsteps, void *stream)
{
    if (!b || nsteps < 0) return NS_ERR_ARG;
    hipStream_t caller = (hipStream_t)stream;
    while (nsteps > 0) {
        const std::vector<int> order = stepping_order(b);
        if (order.empty()) break;
        // steps for which the stepping set stays the same
        int32_t k = nsteps;
        for (int i : order) k = std::min(k, (int32_t)b->m[i].steps_left);
        int32_t eager = k;
        if (b->graphs && k >= kGraphSteps) {
            // whole graphs of kGraphSteps steps on the origin stream, ordered
            // between the caller's earlier and later work
            if (!b->gexec) NS_HIP_OK(capture_steps(b, order));
            NS_HIP_OK(hipEventRecord(b->gin, caller));
            NS_HIP_OK(hipStreamWaitEvent(b->origin, b->gin, 0));
            for (int32_t r = 0; r + kGraphSteps <= k; r += kGraphSteps)
                NS_HIP_OK(hipGraphLaunch(b->gexec, b->origin));
            NS_HIP_OK(hipEventRecord(b->gout, b->origin));
            NS_HIP_OK(hipStreamWaitEvent(caller, b->gout, 0));
            eager = k % kGraphSteps;
        }
        if (eager > 0) NS_HIP_OK(enqueue_steps(b, order, eager, caller));
        bool finished = false;
        for (int i : order) {
            Member &m = b->m[i];
            m.steps_left -= k;
            m.steps_done += k;
            finished = finished || m.steps_left == 0;
        }
        if (finished) drop_graph(b);   // the stepping set changes
        nsteps -= k;
    }
    return NS_OK;
}

ns_status ns_batch_set_graphs(ns_batch *b, int32_t enable)
{
    if (!b || (enable != 0 && enable != 1)) return NS_ERR_ARG;
    if (enable && !b->origin) {
        if (hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->gin, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->gout, hipEventDisableTiming) != hipSuccess)
            return NS_ERR_DEVICE;
    }
    if (!enable) drop_graph(b);
    b->graphs = enable != 0;
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
