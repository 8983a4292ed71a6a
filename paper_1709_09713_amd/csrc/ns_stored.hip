// ns_stored.hip -- the stored-derivative (baseline, BL) algorithm class.
//
// As in the baseline-algorithm section: the primitive variables and every
// product that is differentiated are first written to temporary arrays,
// then each derivative of the governing equations is computed by its own
// stencil sweep (one launch per function, direction and order, like the
// listing's derx subroutine) and stored in its own global work array, and
// finally a pointwise kernel assembles the residual from those arrays.
// Derivative census: 42 first derivatives, 12 second derivatives and the
// 6 mixed derivatives d/dx_i (d u_k/dx_k), i != k, taken as first
// derivatives of the stored velocity-gradient arrays: 60 arrays.
#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

// Work-array layout (units of N doubles).
enum {
    W_U = 0, W_V, W_W, W_P, W_T,          // primitives
    W_MU = 5,                             // m_i u_j, 9 arrays, index 3 i + j
    W_EU = 14,                            // rhoE u_j, 3
    W_PU = 17,                            // p u_j, 3
    W_D = 20,                             // 60 derivative arrays follow
    W_TOTAL = 80
};
// Derivative-array indices (relative to W_D).
enum {
    D_RHO = 0,    // d rho / dx_j                      (3)
    D_M = 3,      // d m_i / dx_j,     3 i + j         (9)
    D_U = 12,     // d u_i / dx_j,     3 i + j         (9)
    D_MU = 21,    // d (m_i u_j) / dx_j, 3 i + j       (9)
    D_E = 30,     // d rhoE / dx_j                     (3)
    D_EU = 33,    // d (rhoE u_j) / dx_j               (3)
    D_PU = 36,    // d (p u_j) / dx_j                  (3)
    D_P = 39,     // d p / dx_i                        (3)
    D2_U = 42,    // d2 u_i / dx_j^2,  3 i + j         (9)
    D2_T = 51,    // d2 T / dx_j^2                     (3)
    D_MIX = 54,   // d/dx_i (d u_k / dx_k), i != k     (6)
    D_COUNT = 60
};

size_t stored_workspace_doubles(const Consts &c) { return (size_t)W_TOTAL * (size_t)c.N; }

__global__ void bl_primitives_kernel(Consts c, const double *__restrict__ Q, double *__restrict__ w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.N) return;
    const int64_t N = c.N;
    const double rho = Q[i], m0 = Q[N + i], m1 = Q[2 * N + i], m2 = Q[3 * N + i], E = Q[4 * N + i];
    const double u = m0 / rho, v = m1 / rho, ww = m2 / rho;
    const double p = c.gm1 * (E - 0.5 * (m0 * u + m1 * v + m2 * ww));
    w[W_U * N + i] = u;
    w[W_V * N + i] = v;
    w[W_W * N + i] = ww;
    w[W_P * N + i] = p;
    w[W_T * N + i] = c.gM2 * p / rho;
}

__global__ void bl_products_kernel(Consts c, const double *__restrict__ Q, double *__restrict__ w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.N) return;
    const int64_t N = c.N;
    const double u[3] = {w[W_U * N + i], w[W_V * N + i], w[W_W * N + i]};
    const double p = w[W_P * N + i], E = Q[4 * N + i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double m = Q[(1 + a) * N + i];
#pragma unroll
        for (int j = 0; j < 3; ++j) w[(W_MU + 3 * a + j) * N + i] = m * u[j];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        w[(W_EU + j) * N + i] = E * u[j];
        w[(W_PU + j) * N + i] = p * u[j];
    }
}

// One derivative sweep: out = D_dir f (order 1, eq. fd) or D2_dir f (order 2,
// eq. sd), periodic.  Block 64 x 4 over (x, y), one z plane per grid z.
__global__ void __launch_bounds__(256)
bl_deriv_kernel(Consts c, const double *__restrict__ f, double *__restrict__ out, int dir, int order)
{
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= c.nx || j >= c.ny) return;
    const int64_t idx = (int64_t)k * c.nxy + (int64_t)j * c.nx + i;
    int co, n;
    int64_t stride;
    if (dir == 0) { co = i; n = c.nx; stride = 1; }
    else if (dir == 1) { co = j; n = c.ny; stride = c.nx; }
    else { co = k; n = c.nz; stride = c.nxy; }
    const double fm2 = f[idx + (int64_t)(wrap1(co - 2, n) - co) * stride];
    const double fm1 = f[idx + (int64_t)(wrap1(co - 1, n) - co) * stride];
    const double fp1 = f[idx + (int64_t)(wrap1(co + 1, n) - co) * stride];
    const double fp2 = f[idx + (int64_t)(wrap1(co + 2, n) - co) * stride];
    out[idx] = order == 1 ? c.c1[dir] * d1u(fm2, fm1, fp1, fp2)
                          : c.c2[dir] * d2u(fm2, fm1, f[idx], fp1, fp2);
}

// Residual assembled pointwise from the stored derivative arrays.
__global__ void bl_residual_kernel(Consts c, const double *__restrict__ Q, const double *__restrict__ w,
                                   double *__restrict__ R)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.N) return;
    const int64_t N = c.N;
    const double *D = w + (int64_t)W_D * N;
#define DA(k) D[(int64_t)(k) * N + i]
    const double rho = Q[i], E = Q[4 * N + i];
    const double m[3] = {Q[N + i], Q[2 * N + i], Q[3 * N + i]};
    const double u[3] = {w[W_U * N + i], w[W_V * N + i], w[W_W * N + i]};
    double G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) G[a][j] = DA(D_U + 3 * a + j);
    const double div = G[0][0] + G[1][1] + G[2][2];

    double r = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) r += DA(D_M + 3 * j + j) + rho * G[j][j] + u[j] * DA(D_RHO + j);
    R[i] = -0.5 * r;

    // viscous: lap u_i + (1/3)(d2 u_i/dx_i^2 + sum_{k != i} d/dx_i du_k/dx_k)
    double V[3];
    const int mix[3][2] = {{0, 1}, {2, 3}, {4, 5}};   // (i, k) pairs in D_MIX order
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double lap = DA(D2_U + 3 * a + 0) + DA(D2_U + 3 * a + 1) + DA(D2_U + 3 * a + 2);
        V[a] = lap + (DA(D2_U + 3 * a + a) + DA(D_MIX + mix[a][0]) + DA(D_MIX + mix[a][1])) / 3.0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double cv = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) cv += DA(D_MU + 3 * a + j) + m[a] * G[j][j] + u[j] * DA(D_M + 3 * a + j);
        R[(1 + a) * N + i] = -0.5 * cv - DA(D_P + a) + c.inv_re * V[a];
    }
    double ce = 0.0, pw = 0.0, ht = 0.0, wk = 0.0, phi = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        ce += DA(D_EU + j) + E * G[j][j] + u[j] * DA(D_E + j);
        pw += DA(D_PU + j);
        ht += DA(D2_T + j);
        wk += u[j] * V[j];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) phi += G[a][j] * (G[a][j] + G[j][a]);
    phi -= (2.0 / 3.0) * div * div;
    R[4 * N + i] = -0.5 * ce - pw + c.inv_re * (wk + phi) + c.kappa * ht;
#undef DA
}

__global__ void rk_update_kernel(int64_t n5, const double *__restrict__ R, const double *__restrict__ acc_in,
                                 double *__restrict__ acc_out, double *__restrict__ qout, double a_dt,
                                 double b_dt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n5) return;
    const double a = acc_in[i], r = R[i];
    qout[i] = a + a_dt * r;
    if (acc_out) acc_out[i] = a + b_dt * r;
}

hipError_t launch_rk_update(const Consts &c, const double *R, const double *acc_in, double *acc_out,
                            double *qout, double a_dt, double b_dt, hipStream_t st)
{
    const int64_t n5 = 5 * c.N;
    hipLaunchKernelGGL(rk_update_kernel, dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, n5, R,
                       acc_in, acc_out, qout, a_dt, b_dt);
    return hipGetLastError();
}

static hipError_t deriv(const Consts &c, const double *f, double *out, int dir, int order, hipStream_t st)
{
    dim3 grid((c.nx + 63) / 64, (c.ny + 3) / 4, c.nz);
    hipLaunchKernelGGL(bl_deriv_kernel, grid, dim3(64, 4, 1), 0, st, c, f, out, dir, order);
    return hipGetLastError();
}

hipError_t stored_residual(const Consts &c, const double *Q, double *R, double *w, hipStream_t st)
{
    const int64_t N = c.N;
    const dim3 pg((unsigned)((N + 255) / 256)), pb(256);
    hipLaunchKernelGGL(bl_primitives_kernel, pg, pb, 0, st, c, Q, w);
    hipLaunchKernelGGL(bl_products_kernel, pg, pb, 0, st, c, Q, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double *D = w + (int64_t)W_D * N;
    auto arr = [&](int k) { return D + (int64_t)k * N; };
    const double *rho = Q, *E = Q + 4 * N;
    for (int j = 0; j < 3 && e == hipSuccess; ++j) {
        e = deriv(c, rho, arr(D_RHO + j), j, 1, st);
        for (int a = 0; a < 3 && e == hipSuccess; ++a) {
            e = deriv(c, Q + (1 + a) * N, arr(D_M + 3 * a + j), j, 1, st);
            if (e == hipSuccess) e = deriv(c, w + (W_U + a) * N, arr(D_U + 3 * a + j), j, 1, st);
            if (e == hipSuccess) e = deriv(c, w + (W_MU + 3 * a + j) * N, arr(D_MU + 3 * a + j), j, 1, st);
            if (e == hipSuccess) e = deriv(c, w + (W_U + a) * N, arr(D2_U + 3 * a + j), j, 2, st);
        }
        if (e == hipSuccess) e = deriv(c, E, arr(D_E + j), j, 1, st);
        if (e == hipSuccess) e = deriv(c, w + (W_EU + j) * N, arr(D_EU + j), j, 1, st);
        if (e == hipSuccess) e = deriv(c, w + (W_PU + j) * N, arr(D_PU + j), j, 1, st);
        if (e == hipSuccess) e = deriv(c, w + W_P * N, arr(D_P + j), j, 1, st);
        if (e == hipSuccess) e = deriv(c, w + W_T * N, arr(D2_T + j), j, 2, st);
    }
    // mixed: d/dx_i of the stored du_k/dx_k, (i, k) in D_MIX order
    const int pairs[6][2] = {{0, 1}, {0, 2}, {1, 0}, {1, 2}, {2, 0}, {2, 1}};
    for (int q = 0; q < 6 && e == hipSuccess; ++q) {
        const int i = pairs[q][0], k = pairs[q][1];
        e = deriv(c, arr(D_U + 3 * k + k), arr(D_MIX + q), i, 1, st);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bl_residual_kernel, pg, pb, 0, st, c, Q, w, R);
    return hipGetLastError();
}

}  // namespace ns
