// ns_probe.hip -- the memory traffic of one fused Runge-Kutta stage without
// its stencil arithmetic.
//
// A stage of the fused class (generic-algorithm figure: evaluate R,
// Q^{k+1} = Q_acc + a_k dt R, Q_acc += b_k dt R) must read its input
// field set and write its output, plus read and/or write the accumulator:
//   stage 1: read Q^n,              write Q^1 and Q_acc   (120 B/point FP64)
//   stage 2: read Q^1 and Q_acc,    write Q^2 and Q_acc   (160 B/point)
//   stage 3: read Q^2 and Q_acc,    write Q^{n+1}         (120 B/point)
// This kernel moves exactly those bytes over the same buffers (one point's
// five fields per lane pair, 16-byte accesses, stage outputs and the
// accumulator non-temporal as in the stage kernels) with a pointwise
// update in place of the residual.  Its rate is what the memory system
// delivers for the stage's access pattern: the achievable ceiling of the
// stage kernel's HBM roofline.
#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

namespace {

typedef double d2_t __attribute__((ext_vector_type(2)));

// Each lane moves two 16-byte chunks per iteration (all loads issued before
// the stores); 64 blocks of 256 lanes per compute unit keep enough bytes in
// flight (the fastest of the shapes measured: 8-64 blocks per CU, one to
// four chunks per lane, non-temporal or cached accesses, 4.7-5.2 TB/s).
// An odd count leaves one double after the last pair; the first lane of
// block 0 moves it.
template <int MODE>
__global__ void __launch_bounds__(256) stream_stage_kernel(int64_t n5, const d2_t *__restrict__ qin,
                                                           const d2_t *__restrict__ acc_in,
                                                           d2_t *__restrict__ acc_out,
                                                           d2_t *__restrict__ qout, double a, double b)
{
    const int64_t npairs = n5 / 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + stride < npairs; i += 2 * stride) {
        const d2_t q0 = qin[i], q1 = qin[i + stride];
        const d2_t a0 = (MODE == 1) ? q0 : __builtin_nontemporal_load(acc_in + i);
        const d2_t a1 = (MODE == 1) ? q1 : __builtin_nontemporal_load(acc_in + i + stride);
        __builtin_nontemporal_store(a0 + a * q0, qout + i);
        __builtin_nontemporal_store(a1 + a * q1, qout + i + stride);
        if (MODE != 3) {
            __builtin_nontemporal_store(a0 + b * q0, acc_out + i);
            __builtin_nontemporal_store(a1 + b * q1, acc_out + i + stride);
        }
    }
    for (; i < npairs; i += stride) {
        const d2_t q = qin[i];
        const d2_t acc = (MODE == 1) ? q : __builtin_nontemporal_load(acc_in + i);
        __builtin_nontemporal_store(acc + a * q, qout + i);
        if (MODE != 3) __builtin_nontemporal_store(acc + b * q, acc_out + i);
    }
    if ((n5 & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t k = n5 - 1;
        const double q = ((const double *)qin)[k];
        const double acc = (MODE == 1) ? q : ((const double *)acc_in)[k];
        ((double *)qout)[k] = acc + a * q;
        if (MODE != 3) ((double *)acc_out)[k] = acc + b * q;
    }
}

}  // namespace

hipError_t launch_stream_stage(int stage, int64_t n5, const double *qin, const double *acc_in,
                               double *acc_out, double *qout, hipStream_t st)
{
    const int64_t npairs = n5 / 2;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    int64_t blocks = (int64_t)cus * 64;
    const int64_t need = (npairs + 255) / 256;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    const d2_t *q = (const d2_t *)qin;
    const d2_t *ai = (const d2_t *)acc_in;
    d2_t *ao = (d2_t *)acc_out;
    d2_t *qo = (d2_t *)qout;
    switch (stage) {
    case 1: hipLaunchKernelGGL(stream_stage_kernel<1>, dim3(blocks), dim3(256), 0, st, n5, q, ai, ao, qo, 0.5, 0.25); break;
    case 2: hipLaunchKernelGGL(stream_stage_kernel<2>, dim3(blocks), dim3(256), 0, st, n5, q, ai, ao, qo, 0.5, 0.25); break;
    case 3: hipLaunchKernelGGL(stream_stage_kernel<3>, dim3(blocks), dim3(256), 0, st, n5, q, ai, ao, qo, 0.5, 0.25); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ns
