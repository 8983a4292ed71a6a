// ns_rs.hip -- the intermediate-storage algorithm class (RS / SS of the
// algorithms section): only the nine velocity-gradient components
// du_i/dx_j are kept in global arrays, every other derivative is evaluated
// inline at the point that needs it.
//
// Per RK stage: rs_gradient_kernel evaluates the nine gradients from the
// conserved variables at the first-derivative taps (u_i = m_i / rho formed
// per tap) and stores them; rs_stage_kernel then evaluates the residual of
// the governing-equations section at each point -- convective, pressure and
// heat-conduction derivatives from the conserved variables at their taps,
// the velocity gradient, divergence and dissipation from the stored arrays,
// the mixed viscous derivatives d/dx_i (du_k/dx_k) as first derivatives of
// the stored diagonal gradients along x_i -- and applies the low-storage RK
// update of the generic-algorithm figure in the same pass.  FP64 only.
#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

namespace {

constexpr int RS_BX = 64, RS_BY = 4;

// Offsets of the four taps of direction d around (i, j, k), periodic.
struct Taps {
    int64_t m2, m1, p1, p2;
};

__device__ __forceinline__ Taps taps(const Consts &c, int i, int j, int k, int d)
{
    int co, n;
    int64_t stride;
    if (d == 0) { co = i; n = c.nx; stride = 1; }
    else if (d == 1) { co = j; n = c.ny; stride = c.nx; }
    else { co = k; n = c.nz; stride = c.nxy; }
    Taps t;
    t.m2 = (int64_t)(wrap1(co - 2, n) - co) * stride;
    t.m1 = (int64_t)(wrap1(co - 1, n) - co) * stride;
    t.p1 = (int64_t)(wrap1(co + 1, n) - co) * stride;
    t.p2 = (int64_t)(wrap1(co + 2, n) - co) * stride;
    return t;
}

// Primitive values at one stencil tap, from the conserved state.  Every
// point that uses a tap recomputes them, so they are evaluated without
// multiply-add contraction: each value is rounded once, identically in
// every context, and the periodic sums of the flux differences telescope
// exactly as with values stored once (discrete conservation).
struct TapVals {
    double rho, m[3], E, u[3], p, T;
};

__device__ __forceinline__ TapVals tap_vals(const Consts &c, const double *__restrict__ Q, int64_t at)
{
#pragma clang fp contract(off)
    const int64_t N = c.N;
    TapVals v;
    v.rho = Q[at];
    v.m[0] = Q[N + at];
    v.m[1] = Q[2 * N + at];
    v.m[2] = Q[3 * N + at];
    v.E = Q[4 * N + at];
    const double inv = 1.0 / v.rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) v.u[a] = v.m[a] * inv;
    v.p = c.gm1 * (v.E - 0.5 * (v.m[0] * v.u[0] + v.m[1] * v.u[1] + v.m[2] * v.u[2]));
    v.T = c.gM2 * v.p * inv;
    return v;
}

// Product of two tap values, rounded once (see tap_vals).
__device__ __forceinline__ double tap_prod(double a, double b)
{
#pragma clang fp contract(off)
    return a * b;
}

__device__ __forceinline__ double tap_velocity(double m, double inv)
{
#pragma clang fp contract(off)
    return m * inv;
}

__global__ void __launch_bounds__(RS_BX * RS_BY)
rs_gradient_kernel(Consts c, const double *__restrict__ Q, double *__restrict__ G)
{
    const int i = blockIdx.x * RS_BX + threadIdx.x, j = blockIdx.y * RS_BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= c.nx || j >= c.ny) return;
    const int64_t idx = (int64_t)k * c.nxy + (int64_t)j * c.nx + i;
    const int64_t N = c.N;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const Taps t = taps(c, i, j, k, d);
        const int64_t at[4] = {idx + t.m2, idx + t.m1, idx + t.p1, idx + t.p2};
        double u[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double inv = 1.0 / Q[at[q]];
#pragma unroll
            for (int a = 0; a < 3; ++a) u[q][a] = tap_velocity(Q[(1 + a) * N + at[q]], inv);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
            G[(3 * a + d) * N + idx] = c.c1[d] * d1u(u[0][a], u[1][a], u[2][a], u[3][a]);
    }
}

struct RsArgs {
    const double *qin;
    const double *G;
    const double *acc_in;
    double *acc_out;
    double *qout;
    double *rout;
    double a_dt, b_dt;
    int mode;   // 0 = residual only, 1..3 = RK stage
};

__global__ void __launch_bounds__(RS_BX * RS_BY) rs_stage_kernel(Consts c, RsArgs s)
{
    const int i = blockIdx.x * RS_BX + threadIdx.x, j = blockIdx.y * RS_BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= c.nx || j >= c.ny) return;
    const int64_t idx = (int64_t)k * c.nxy + (int64_t)j * c.nx + i;
    const int64_t N = c.N;
    const double *__restrict__ Q = s.qin;
    const double *__restrict__ G = s.G;

    const TapVals o = tap_vals(c, Q, idx);
    double g[3][3];   // g[a][d] = du_a / dx_d (stored)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[a][d] = G[(3 * a + d) * N + idx];
    const double div = g[0][0] + g[1][1] + g[2][2];

    // Derivatives recomputed inline from the taps of each direction d.
    double dm_sum = 0.0;                 // sum_d D_d m_d
    double urho = 0.0, uE = 0.0;         // sum_d u_d D_d rho, sum_d u_d D_d rhoE
    double dEu = 0.0, dpu = 0.0;         // sum_d D_d (rhoE u_d), sum_d D_d (p u_d)
    double lapT = 0.0;                   // sum_d D2_d T
    double dmu[3] = {0.0, 0.0, 0.0};     // sum_d D_d (m_a u_d)
    double udm[3] = {0.0, 0.0, 0.0};     // sum_d u_d D_d m_a
    double lapu[3] = {0.0, 0.0, 0.0};    // sum_d D2_d u_a
    double d2ii[3];                      // D2_a u_a
    double dp[3];                        // D_a p
    double mixv[3];                      // sum_{k != a} D_a (du_k/dx_k)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const Taps t = taps(c, i, j, k, d);
        const TapVals a = tap_vals(c, Q, idx + t.m2), b = tap_vals(c, Q, idx + t.m1);
        const TapVals e = tap_vals(c, Q, idx + t.p1), f = tap_vals(c, Q, idx + t.p2);
        const double c1 = c.c1[d], c2 = c.c2[d];
#define D1(x) (c1 * d1u(a.x, b.x, e.x, f.x))
#define D2(x) (c2 * d2u(a.x, b.x, o.x, e.x, f.x))
        dm_sum += D1(m[d]);
        urho += o.u[d] * D1(rho);
        uE += o.u[d] * D1(E);
        dEu += c1 * d1u(tap_prod(a.E, a.u[d]), tap_prod(b.E, b.u[d]), tap_prod(e.E, e.u[d]),
                        tap_prod(f.E, f.u[d]));
        dpu += c1 * d1u(tap_prod(a.p, a.u[d]), tap_prod(b.p, b.u[d]), tap_prod(e.p, e.u[d]),
                        tap_prod(f.p, f.u[d]));
        lapT += D2(T);
        dp[d] = D1(p);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            dmu[q] += c1 * d1u(tap_prod(a.m[q], a.u[d]), tap_prod(b.m[q], b.u[d]),
                               tap_prod(e.m[q], e.u[d]), tap_prod(f.m[q], f.u[d]));
            udm[q] += o.u[d] * D1(m[q]);
            const double d2 = D2(u[q]);
            lapu[q] += d2;
            if (q == d) d2ii[q] = d2;
        }
#undef D1
#undef D2
        // mixed: D_d of the stored diagonal gradients of the other directions
        double mx = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (q == d) continue;
            const double *Gq = G + (int64_t)(4 * q) * N;   // du_q / dx_q
            mx += c1 * d1u(Gq[idx + t.m2], Gq[idx + t.m1], Gq[idx + t.p1], Gq[idx + t.p2]);
        }
        mixv[d] = mx;
    }

    double R[5];
    R[0] = -0.5 * (dm_sum + o.rho * div + urho);
    double V[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        V[a] = lapu[a] + (d2ii[a] + mixv[a]) / 3.0;
        R[1 + a] = -0.5 * (dmu[a] + o.m[a] * div + udm[a]) - dp[a] + c.inv_re * V[a];
    }
    double phi = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) phi += g[a][d] * (g[a][d] + g[d][a]);
    phi -= (2.0 / 3.0) * div * div;
    const double work = o.u[0] * V[0] + o.u[1] * V[1] + o.u[2] * V[2];
    R[4] = -0.5 * (dEu + o.E * div + uE) - dpu + c.inv_re * (work + phi) + c.kappa * lapT;

    if (s.mode == 0) {
#pragma unroll
        for (int f = 0; f < 5; ++f) s.rout[f * N + idx] = R[f];
        return;
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const double acc = (s.mode == 1) ? Q[f * N + idx] : s.acc_in[f * N + idx];
        s.qout[f * N + idx] = acc + s.a_dt * R[f];
        if (s.mode < 3) s.acc_out[f * N + idx] = acc + s.b_dt * R[f];
    }
}

dim3 rs_grid(const Consts &c) { return dim3((c.nx + RS_BX - 1) / RS_BX, (c.ny + RS_BY - 1) / RS_BY, c.nz); }

}  // namespace

size_t rs_workspace_doubles(const Consts &c) { return 9 * (size_t)c.N; }

hipError_t rs_stage(const Consts &c, const double *qin, double *G, const double *acc_in, double *acc_out,
                    double *qout, double *rout, double a_dt, double b_dt, int mode, hipStream_t st)
{
    hipLaunchKernelGGL(rs_gradient_kernel, rs_grid(c), dim3(RS_BX, RS_BY, 1), 0, st, c, qin, G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    RsArgs a;
    a.qin = qin;
    a.G = G;
    a.acc_in = acc_in;
    a.acc_out = acc_out;
    a.qout = qout;
    a.rout = rout;
    a.a_dt = a_dt;
    a.b_dt = b_dt;
    a.mode = mode;
    hipLaunchKernelGGL(rs_stage_kernel, rs_grid(c), dim3(RS_BX, RS_BY, 1), 0, st, c, a);
    return hipGetLastError();
}

}  // namespace ns
