// ns_noalloc.hip -- rk3_step of the fused class for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// rk3_step takes its scratch (RK accumulator, two stage buffers, diagnostic
// partials) from a caller-provided workspace.  rk3_step_noalloc takes it
// from `scratch`, a static device array of kScratchBytes that every GPU the
// library runs on holds until the process ends.  In host code the array's
// name is only a host-side handle: its device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and kept per
// device, and only that address is passed to the kernels.  The entry point
// allocates nothing and calls exactly rk3_step's kernels on that workspace.
// Nothing in it has to start at zero: every stage writes a buffer before a
// later stage reads it, and stage 1 writes every diagnostic partial that the
// reduction reads.  All calls on one GPU share its array, so calls that
// overlap on one GPU (other streams, other threads) race.
#include <cmath>
#include <mutex>

#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

// 64 MiB: the FP64 fused workspace is about 120 B per grid point, so grids
// up to about 550,000 points (80^3) fit; FP32 storage up to about 80^3 too
// (the stage buffers are float but the accumulator stays double).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, looked up on the first
// call made there.  nullptr if the device cannot be queried or the lookup
// fails.
static void *scratch_on_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace ns

using namespace ns;

extern "C" {

size_t ns_noalloc_scratch_bytes(void) { return kScratchBytes; }

ns_status rk3_step_noalloc(const ns_params *p, ns_precision prec, double dt, int32_t nsteps,
                           double *state, ns_diag *diag_dev, void *stream)
{
    // everything rk3_step checks, and the size limit, before the device is
    // touched
    ns_status st = validate_params(p);
    if (st != NS_OK) return st;
    if (prec != NS_FP64 && prec != NS_FP32_STORE) return NS_ERR_ARG;
    const size_t need = ns_workspace_bytes(p, NS_ALGO_FUSED, prec);
    if (need > kScratchBytes) return NS_ERR_WORKSPACE;
    if (!state || ((uintptr_t)state & 15) != 0) return NS_ERR_ARG;
    if (diag_dev && ((uintptr_t)diag_dev & 7) != 0) return NS_ERR_ARG;
    if (!std::isfinite(dt) || !(dt > 0.0) || nsteps < 0) return NS_ERR_ARG;
    if (nsteps == 0) return NS_OK;
    void *work = scratch_on_current_device();
    if (!work) return NS_ERR_DEVICE;
    FusedPlan f;
    st = make_fused_plan(p, prec, -1, 0, state, work, kScratchBytes, &f);
    if (st != NS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    for (int32_t step = 0; step < nsteps; ++step)
        NS_HIP_OK(enqueue_fused_step(f, dt, diag_dev ? diag_dev + step : nullptr, s));
    return NS_OK;
}

}  // extern "C"
