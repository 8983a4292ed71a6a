// ns_diag.hip -- Taylor-Green initial state and the FP64 diagnostics.
//
// tgv_init writes the initial condition of the results section.
// The diagnostics are the kinetic-energy / enstrophy quantities of the
// validation data set that the results section compares against, plus the
// conserved totals: per-block partial sums (wave64 shuffle reduction, then
// LDS across waves) and a one-block final pass in a fixed order, so the
// result is bitwise reproducible for a given grid.
#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

__global__ void tgv_init_kernel(Consts c, double gamma, double mach, double *__restrict__ Q)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= c.N) return;
    const int i = (int)(idx % c.nx);
    const int j = (int)((idx / c.nx) % c.ny);
    const int k = (int)(idx / c.nxy);
    // x / L with L = length / (2 pi) and h = length / n: x / L = 2 pi i / n
    const double two_pi = 6.283185307179586476925286766559;
    const double x = (double)i * (two_pi / c.nx);
    const double y = (double)j * (two_pi / c.ny);
    const double z = (double)k * (two_pi / c.nz);
    double sx, cx, sy, cy, sz, cz;
    sincos(x, &sx, &cx);
    sincos(y, &sy, &cy);
    sincos(z, &sz, &cz);
    (void)sz;
    const double u = sx * cy * cz;
    const double v = -cx * sy * cz;
    const double gM2 = gamma * mach * mach;
    const double p = 1.0 / gM2 + (cos(2.0 * x) + cos(2.0 * y)) * (2.0 + cos(2.0 * z)) / 16.0;
    const double rho = gM2 * p;
    const int64_t N = c.N;
    Q[idx] = rho;
    Q[N + idx] = rho * u;
    Q[2 * N + idx] = rho * v;
    Q[3 * N + idx] = 0.0;
    Q[4 * N + idx] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v);
}

hipError_t launch_tgv_init(const Consts &c, const ns_params *p, double *state, hipStream_t st)
{
    hipLaunchKernelGGL(tgv_init_kernel, dim3((unsigned)((c.N + 255) / 256)), dim3(256), 0, st, c,
                       p->gamma, p->mach, state);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagnostics partials: one block of 256 threads per (x-row strip of 256
// points); each thread handles one point, vorticity from fd stencils of
// u = m / rho evaluated at the taps.
constexpr int kDiagThreads = 256;

int64_t diag_num_blocks(const Consts &c) { return (c.N + kDiagThreads - 1) / kDiagThreads; }

__device__ __forceinline__ double vel(const double *Q, int64_t N, int64_t i, int comp)
{
    return Q[(1 + comp) * N + i] / Q[i];
}

__global__ void __launch_bounds__(kDiagThreads)
diag_partial_kernel(Consts c, const double *__restrict__ Q, double *__restrict__ partial)
{
    __shared__ double red[kDiagThreads / 64][kDiag];
    const int64_t idx = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x;
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    if (idx < c.N) {
        const int64_t N = c.N;
        const int i = (int)(idx % c.nx);
        const int j = (int)((idx / c.nx) % c.ny);
        const int k = (int)(idx / c.nxy);
        const int co[3] = {i, j, k};
        const int nn[3] = {c.nx, c.ny, c.nz};
        const int64_t st[3] = {1, c.nx, c.nxy};
        // G[a][d] = d u_a / d x_d
        double G[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t im2 = idx + (int64_t)(wrap1(co[d] - 2, nn[d]) - co[d]) * st[d];
            const int64_t im1 = idx + (int64_t)(wrap1(co[d] - 1, nn[d]) - co[d]) * st[d];
            const int64_t ip1 = idx + (int64_t)(wrap1(co[d] + 1, nn[d]) - co[d]) * st[d];
            const int64_t ip2 = idx + (int64_t)(wrap1(co[d] + 2, nn[d]) - co[d]) * st[d];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                G[a][d] = c.c1[d] * d1u(vel(Q, N, im2, a), vel(Q, N, im1, a), vel(Q, N, ip1, a),
                                        vel(Q, N, ip2, a));
        }
        const double rho = Q[idx];
        const double m0 = Q[N + idx], m1 = Q[2 * N + idx], m2 = Q[3 * N + idx];
        const double ox = G[2][1] - G[1][2], oy = G[0][2] - G[2][0], oz = G[1][0] - G[0][1];
        s[0] = rho;
        s[1] = m0;
        s[2] = m1;
        s[3] = m2;
        s[4] = Q[4 * N + idx];
        s[5] = 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho;
        s[6] = 0.5 * rho * (ox * ox + oy * oy + oz * oz);
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        double v = s[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        s[q] = v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int q = 0; q < 7; ++q) red[wave][q] = s[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 7; ++q) {
            double t = 0.0;
            for (int wv = 0; wv < kDiagThreads / 64; ++wv) t += red[wv][q];
            partial[(int64_t)blockIdx.x * kDiag + q] = t;
        }
        partial[(int64_t)blockIdx.x * kDiag + 7] = 0.0;
    }
}

hipError_t launch_diag_partials(const Consts &c, const double *state, double *partial, hipStream_t st)
{
    hipLaunchKernelGGL(diag_partial_kernel, dim3((unsigned)diag_num_blocks(c)), dim3(kDiagThreads), 0, st,
                       c, state, partial);
    return hipGetLastError();
}

// Fixed-order final reduction: thread t sums partials t, t+256, ... in
// order; then a fixed pairwise tree over the 256 thread sums.
__global__ void __launch_bounds__(256)
diag_finalize_kernel(Consts c, const double *__restrict__ partial, int64_t nblocks, ns_diag *out)
{
    __shared__ double red[256][7];
    const int t = threadIdx.x;
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = t; b < nblocks; b += 256)
#pragma unroll
        for (int q = 0; q < 7; ++q) s[q] += partial[b * kDiag + q];
#pragma unroll
    for (int q = 0; q < 7; ++q) red[t][q] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < 7; ++q) red[t][q] += red[t + w][q];
        __syncthreads();
    }
    if (t == 0) {
        out->mass = c.vol * red[0][0];
        out->momentum[0] = c.vol * red[0][1];
        out->momentum[1] = c.vol * red[0][2];
        out->momentum[2] = c.vol * red[0][3];
        out->energy = c.vol * red[0][4];
        out->kinetic_energy = red[0][5] * c.inv_npts;
        out->enstrophy = red[0][6] * c.inv_npts;
        out->dissipation = 2.0 * out->enstrophy * c.inv_re;
    }
}

hipError_t launch_diag_finalize(const Consts &c, const double *partial, int64_t nblocks, ns_diag *out,
                                hipStream_t st)
{
    hipLaunchKernelGGL(diag_finalize_kernel, dim3(1), dim3(256), 0, st, c, partial, nblocks, out);
    return hipGetLastError();
}

}  // namespace ns
