// ns_fused.hip -- the fused on-the-fly residual + RK3 stage kernel.
//
// This is the minimal-storage algorithm class of the algorithms section
// (RA / SN / SN2): no derivative is written to a global array.  Every
// derivative of the mass, momentum and energy equations (methodology
// section; stencils fd and sd) is evaluated on the fly and accumulated
// straight into the five residual registers of its grid point, and the
// low-storage RK3 update of the generic-algorithm figure is applied in the
// same pass, so a stage reads its input once and writes its outputs once.
//
// MI355X mapping:
//  * A block owns a BX x BY column tile of the (x, y) plane and marches
//    along z through a chunk of planes.  Each plane of the tile plus a
//    radius-2 halo (wrap-around indexing replaces the periodic-boundary
//    pass) is loaded with coalesced x-fastest loads, turned into the
//    primitive variables once per point, and staged in LDS (double
//    buffered, one barrier per plane).  x and y stencil taps are LDS reads.
//  * z taps come from a per-thread register queue holding the thread's own
//    column for planes z-2..z+2.
//  * The in-plane part of the residual at plane z is computed while z is in
//    LDS and carried in registers for two planes until the z taps of z+2
//    arrive.  Mixed derivatives that involve z are taken as z-derivatives of
//    in-plane derivatives (D_x D_z w = D_z D_x w, exact in exact arithmetic),
//    so only three in-plane quantities (D_x u + D_y v, D_x w, D_y w) need a
//    register queue; D_x D_y is a 16-tap LDS stencil.
//  * Stage 1 can also emit the per-block partial sums of the diagnostics of
//    its input state, so the per-step diagnostics cost no extra pass.
//
// Precision: CT is the stencil/residual arithmetic type.  With CT = float
// (FP32 storage) the staged fields are deviations from the uniform
// reference state (rho - 1, rhoE - rhoE_ref, p - p_ref, T - 1); the constant
// parts are applied analytically (stencil coefficients sum to zero), and the
// RK accumulator stays double.
#include <type_traits>

#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

template <typename TIN, typename CT>
__device__ __forceinline__ CT load_dev(const TIN *q, int64_t i, double ref)
{
    if constexpr (std::is_same<CT, double>::value) {
        return q[i];
    } else if constexpr (std::is_same<TIN, double>::value) {
        return (float)(q[i] - ref);
    } else {
        return q[i];
    }
}

template <typename TOUT>
__device__ __forceinline__ void store_q(void *q, int64_t i, double v, double ref)
{
    if constexpr (std::is_same<TOUT, double>::value)
        ((double *)q)[i] = v;
    else
        ((float *)q)[i] = (float)(v - ref);
}

template <int BX, int BY, typename TIN, typename TOUT, typename CT>
__global__ void __launch_bounds__(BX * BY)
fused_stage_kernel(Consts c, StageArgs s)
{
    constexpr bool DEV = std::is_same<CT, float>::value;
    constexpr int HX = BX + 4, HY = BY + 4, HP = HX * HY, NT = BX * BY;
    constexpr int NLOAD = (HP + NT - 1) / NT;
    enum { L_RHO, L_M0, L_M1, L_M2, L_E, L_U, L_V, L_W, L_P, L_T, NF };
    __shared__ CT lds[2][NF][HP];
    __shared__ double red[NT / 64 + 1][kDiag];

    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    const int x0 = blockIdx.x * BX, y0 = blockIdx.y * BY;
    const int z0 = blockIdx.z * s.zchunk;
    const int z1 = min(z0 + s.zchunk, c.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = (gx < c.nx) && (gy < c.ny);
    const int own = (ty + 2) * HX + tx + 2;
    const int64_t N = c.N;
    const TIN *qin = (const TIN *)s.qin;
    const bool want_diag = s.diag_partial != nullptr;

    // Plane offsets of the points this thread loads (fixed for the march).
    int loff[NLOAD];
#pragma unroll
    for (int r = 0; r < NLOAD; ++r) {
        const int idx = tid + r * NT;
        loff[r] = 0;
        if (idx < HP) {
            const int lx = idx % HX, ly = idx / HX;
            int xx = (x0 + lx - 2) % c.nx;
            if (xx < 0) xx += c.nx;
            int yy = (y0 + ly - 2) % c.ny;
            if (yy < 0) yy += c.ny;
            loff[r] = yy * c.nx + xx;
        }
    }

    const CT c1x = (CT)c.c1[0], c1y = (CT)c.c1[1], c1z = (CT)c.c1[2];
    const CT c2x = (CT)c.c2[0], c2y = (CT)c.c2[1], c2z = (CT)c.c2[2];
    const CT inv_re = (CT)c.inv_re, kappa = (CT)c.kappa;
    const CT gm1 = (CT)c.gm1, gM2 = (CT)c.gM2;
    const CT half = CT(0.5), third = CT(1) / CT(3), four3 = CT(4) / CT(3);
    const CT two3 = CT(2) / CT(3);

    CT qv[5][NF];                 // own column, planes zp-4 .. zp
    CT qa[5], qb[5], qc[5];       // D_x u + D_y v, D_x w, D_y w at zp-4 .. zp
    CT pr[3][6];                  // in-plane partial residual + omega_z, zp-2 .. zp
    double dsum[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        qa[q] = qb[q] = qc[q] = CT(0);
#pragma unroll
        for (int f = 0; f < NF; ++f) qv[q][f] = CT(0);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int f = 0; f < 6; ++f) pr[q][f] = CT(0);

    for (int zp = z0 - 2; zp < z1 + 2; ++zp) {
        const int b = (zp - z0) & 1;
        const int zw = wrap1(zp, c.nz);
        const int64_t base = (int64_t)zw * c.nxy;

        // ---- stage plane zp (tile + halo): conserved -> primitives -> LDS
#pragma unroll
        for (int r = 0; r < NLOAD; ++r) {
            const int idx = tid + r * NT;
            if (idx < HP) {
                const int64_t g = base + loff[r];
                const CT rho = load_dev<TIN, CT>(qin, g, c.rho_ref);
                const CT m0 = load_dev<TIN, CT>(qin, g + N, 0.0);
                const CT m1 = load_dev<TIN, CT>(qin, g + 2 * N, 0.0);
                const CT m2 = load_dev<TIN, CT>(qin, g + 3 * N, 0.0);
                const CT E = load_dev<TIN, CT>(qin, g + 4 * N, c.rhoE_ref);
                const CT rhof = DEV ? CT(1) + rho : rho;
                const CT inv = CT(1) / rhof;
                const CT u = m0 * inv, v = m1 * inv, w = m2 * inv;
                const CT p = gm1 * (E - half * (m0 * u + m1 * v + m2 * w));
                // T = gamma M^2 p / rho; as a deviation from T = 1 when the
                // reference state satisfies gamma M^2 p_ref = rho_ref = 1.
                const CT T = DEV ? (gM2 * p - rho) * inv : gM2 * p * inv;
                lds[b][L_RHO][idx] = rho;
                lds[b][L_M0][idx] = m0;
                lds[b][L_M1][idx] = m1;
                lds[b][L_M2][idx] = m2;
                lds[b][L_E][idx] = E;
                lds[b][L_U][idx] = u;
                lds[b][L_V][idx] = v;
                lds[b][L_W][idx] = w;
                lds[b][L_P][idx] = p;
                lds[b][L_T][idx] = T;
            }
        }
        __syncthreads();

#define LV(f, dy, dx) lds[b][f][own + (dy) * HX + (dx)]
#define DX1(f) d1u(LV(f, 0, -2), LV(f, 0, -1), LV(f, 0, 1), LV(f, 0, 2))
#define DY1(f) d1u(LV(f, -2, 0), LV(f, -1, 0), LV(f, 1, 0), LV(f, 2, 0))
#define DX1P(f, g)                                                       \
    d1u(LV(f, 0, -2) * LV(g, 0, -2), LV(f, 0, -1) * LV(g, 0, -1),        \
        LV(f, 0, 1) * LV(g, 0, 1), LV(f, 0, 2) * LV(g, 0, 2))
#define DY1P(f, g)                                                       \
    d1u(LV(f, -2, 0) * LV(g, -2, 0), LV(f, -1, 0) * LV(g, -1, 0),        \
        LV(f, 1, 0) * LV(g, 1, 0), LV(f, 2, 0) * LV(g, 2, 0))
#define DX2(f) d2u(LV(f, 0, -2), LV(f, 0, -1), LV(f, 0, 0), LV(f, 0, 1), LV(f, 0, 2))
#define DY2(f) d2u(LV(f, -2, 0), LV(f, -1, 0), LV(f, 0, 0), LV(f, 1, 0), LV(f, 2, 0))
// D_x applied to D_y f (16 taps), unscaled.
#define DXDY(f)                                                          \
    d1u(d1u(LV(f, -2, -2), LV(f, -1, -2), LV(f, 1, -2), LV(f, 2, -2)),   \
        d1u(LV(f, -2, -1), LV(f, -1, -1), LV(f, 1, -1), LV(f, 2, -1)),   \
        d1u(LV(f, -2, 1), LV(f, -1, 1), LV(f, 1, 1), LV(f, 2, 1)),       \
        d1u(LV(f, -2, 2), LV(f, -1, 2), LV(f, 1, 2), LV(f, 2, 2)))
// D_y applied to D_x f (16 taps), unscaled.
#define DYDX(f)                                                          \
    d1u(d1u(LV(f, -2, -2), LV(f, -2, -1), LV(f, -2, 1), LV(f, -2, 2)),   \
        d1u(LV(f, -1, -2), LV(f, -1, -1), LV(f, -1, 1), LV(f, -1, 2)),   \
        d1u(LV(f, 1, -2), LV(f, 1, -1), LV(f, 1, 1), LV(f, 1, 2)),       \
        d1u(LV(f, 2, -2), LV(f, 2, -1), LV(f, 2, 1), LV(f, 2, 2)))

        // ---- in-plane part at plane zp
        CT cen[NF];
        CT na = CT(0), nb = CT(0), nc = CT(0);
        CT np[6] = {CT(0), CT(0), CT(0), CT(0), CT(0), CT(0)};
        if (active) {
#pragma unroll
            for (int f = 0; f < NF; ++f) cen[f] = LV(f, 0, 0);
            const CT Gxx = c1x * DX1(L_U), Gxy = c1y * DY1(L_U);
            const CT Gyx = c1x * DX1(L_V), Gyy = c1y * DY1(L_V);
            const CT Gzx = c1x * DX1(L_W), Gzy = c1y * DY1(L_W);
            na = Gxx + Gyy;
            nb = Gzx;
            nc = Gzy;
            if (zp >= z0 && zp < z1) {
                const CT rho = cen[L_RHO], E = cen[L_E];
                const CT u = cen[L_U], v = cen[L_V], w = cen[L_W];
                const CT rhof = DEV ? CT(1) + rho : rho;
                const CT a = na;
                // mass: -1/2 (d(rho u_j)/dx_j + rho du_j/dx_j + u_j drho/dx_j), j = x, y
                np[0] = -half * (c1x * DX1(L_M0) + c1y * DY1(L_M1) + rhof * a
                                 + u * (c1x * DX1(L_RHO)) + v * (c1y * DY1(L_RHO)));
                // momentum convection and pressure gradient, j = x, y
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int Lm = L_M0 + i;
                    np[1 + i] = -half * (c1x * DX1P(Lm, L_U) + c1y * DY1P(Lm, L_V)
                                         + cen[Lm] * a + u * (c1x * DX1(Lm))
                                         + v * (c1y * DY1(Lm)));
                }
                np[1] -= c1x * DX1(L_P);
                np[2] -= c1y * DY1(L_P);
                // viscous: d_j tau_ij = lap u_i + (1/3) d_i div u, in-plane parts
                const CT Vx = four3 * (c2x * DX2(L_U)) + c2y * DY2(L_U)
                              + third * (c1x * c1y * DXDY(L_V));
                const CT Vy = c2x * DX2(L_V) + four3 * (c2y * DY2(L_V))
                              + third * (c1x * c1y * DYDX(L_U));
                const CT Vz = c2x * DX2(L_W) + c2y * DY2(L_W);
                np[1] += inv_re * Vx;
                np[2] += inv_re * Vy;
                np[3] += inv_re * Vz;
                // tau_ij du_i/dx_j restricted to terms without a z derivative
                const CT phi = CT(2) * (Gxx * Gxx + Gyy * Gyy) + Gxy * Gxy + Gyx * Gyx
                               + CT(2) * Gxy * Gyx + Gzx * Gzx + Gzy * Gzy;
                // energy: skew convection, pressure work, viscous work,
                // dissipation and heat conduction, j = x, y.  The constant
                // part H_ref * div of the FP32 deviation form is added in
                // double at the end.
                np[4] = -half * (c1x * DX1P(L_E, L_U) + c1y * DY1P(L_E, L_V) + E * a
                                 + u * (c1x * DX1(L_E)) + v * (c1y * DY1(L_E)))
                        - (c1x * DX1P(L_P, L_U) + c1y * DY1P(L_P, L_V))
                        + inv_re * (u * Vx + v * Vy + w * Vz + phi)
                        + kappa * (c2x * DX2(L_T) + c2y * DY2(L_T));
                np[5] = Gyx - Gxy;   // omega_z, for the diagnostics
            }
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) cen[f] = CT(0);
        }
#undef LV
#undef DX1
#undef DY1
#undef DX1P
#undef DY1P
#undef DX2
#undef DY2
#undef DXDY
#undef DYDX

        // ---- advance the register queues
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int f = 0; f < NF; ++f) qv[q][f] = qv[q + 1][f];
            qa[q] = qa[q + 1];
            qb[q] = qb[q + 1];
            qc[q] = qc[q + 1];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) qv[4][f] = cen[f];
        qa[4] = na;
        qb[4] = nb;
        qc[4] = nc;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            pr[0][f] = pr[1][f];
            pr[1][f] = pr[2][f];
            pr[2][f] = np[f];
        }

        // ---- finish plane zf = zp - 2: z derivatives, RK update, output
        const int zf = zp - 2;
        if (active && zf >= z0 && zf < z1) {
#define DZ1(f) d1u(qv[0][f], qv[1][f], qv[3][f], qv[4][f])
#define DZ1P(f, g) \
    d1u(qv[0][f] * qv[0][g], qv[1][f] * qv[1][g], qv[3][f] * qv[3][g], qv[4][f] * qv[4][g])
#define DZ2(f) d2u(qv[0][f], qv[1][f], qv[2][f], qv[3][f], qv[4][f])
            const CT rho = qv[2][L_RHO], E = qv[2][L_E];
            const CT u = qv[2][L_U], v = qv[2][L_V], w = qv[2][L_W];
            const CT rhof = DEV ? CT(1) + rho : rho;
            const CT a = qa[2], bb = qb[2], cc = qc[2];
            const CT Gxz = c1z * DZ1(L_U), Gyz = c1z * DZ1(L_V), Gzz = c1z * DZ1(L_W);
            const CT Da = c1z * d1u(qa[0], qa[1], qa[3], qa[4]);
            const CT Db = c1z * d1u(qb[0], qb[1], qb[3], qb[4]);
            const CT Dc = c1z * d1u(qc[0], qc[1], qc[3], qc[4]);

            CT R[5];
            R[0] = pr[0][0] - half * (c1z * DZ1(L_M2) + rhof * Gzz + w * (c1z * DZ1(L_RHO)));
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int Lm = L_M0 + i;
                R[1 + i] = pr[0][1 + i]
                           - half * (c1z * DZ1P(Lm, L_W) + qv[2][Lm] * Gzz
                                     + w * (c1z * DZ1(Lm)));
            }
            R[3] -= c1z * DZ1(L_P);
            const CT Vx = c2z * DZ2(L_U) + third * Db;
            const CT Vy = c2z * DZ2(L_V) + third * Dc;
            const CT Vz = four3 * (c2z * DZ2(L_W)) + third * Da;
            R[1] += inv_re * Vx;
            R[2] += inv_re * Vy;
            R[3] += inv_re * Vz;
            const CT div = a + Gzz;
            const CT phi = Gxz * Gxz + Gyz * Gyz + CT(2) * Gzz * Gzz
                           + CT(2) * (Gxz * bb + Gyz * cc) - two3 * div * div;
            R[4] = pr[0][4]
                   - half * (c1z * DZ1P(L_E, L_W) + E * Gzz + w * (c1z * DZ1(L_E)))
                   - c1z * DZ1P(L_P, L_W)
                   + inv_re * (u * Vx + v * Vy + w * Vz + phi)
                   + kappa * (c2z * DZ2(L_T));

            double Rd[5];
#pragma unroll
            for (int f = 0; f < 5; ++f) Rd[f] = (double)R[f];
            if constexpr (DEV) Rd[4] -= c.H_ref * ((double)a + (double)Gzz);

            const int64_t pidx = (int64_t)zf * c.nxy + (int64_t)gy * c.nx + gx;
            if (s.mode == 0) {
#pragma unroll
                for (int f = 0; f < 5; ++f) s.rout[f * N + pidx] = Rd[f];
            } else {
                const double ref[5] = {c.rho_ref, 0.0, 0.0, 0.0, c.rhoE_ref};
                double acc[5];
                if (s.mode == 1) {
                    if constexpr (DEV) {
                        // exact double state: re-read (TIN is double in stage 1)
#pragma unroll
                        for (int f = 0; f < 5; ++f)
                            acc[f] = ((const double *)s.qin)[f * N + pidx];
                    } else {
#pragma unroll
                        for (int f = 0; f < 5; ++f) acc[f] = (double)qv[2][L_RHO + f];
                    }
                    if (want_diag) {
                        // diagnostics of the stage input (the state at step
                        // start): conserved totals from the exact double
                        // state, kinetic energy and enstrophy from the staged
                        // primitives and gradients
                        const CT ox = cc - Gyz, oy = Gxz - bb, oz = pr[0][5];
#pragma unroll
                        for (int f = 0; f < 5; ++f) dsum[f] += acc[f];
                        dsum[5] += 0.5 * (acc[1] * (double)u + acc[2] * (double)v + acc[3] * (double)w);
                        dsum[6] += 0.5 * (double)rhof * ((double)ox * (double)ox + (double)oy * (double)oy
                                                         + (double)oz * (double)oz);
                    }
                } else {
#pragma unroll
                    for (int f = 0; f < 5; ++f) acc[f] = s.acc_in[f * N + pidx];
                }
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    store_q<TOUT>(s.qout, f * N + pidx, acc[f] + s.a_dt * Rd[f], ref[f]);
                    if (s.mode < 3) s.acc_out[f * N + pidx] = acc[f] + s.b_dt * Rd[f];
                }
            }
#undef DZ1
#undef DZ1P
#undef DZ2
        }
    }

    if (want_diag) {
        // block reduction of the diagnostic partial sums, fixed order
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            double vsum = dsum[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) vsum += __shfl_xor(vsum, off, 64);
            dsum[k] = vsum;
        }
        const int lane = tid & 63, wave = tid >> 6;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 7; ++k) red[wave][k] = dsum[k];
        }
        __syncthreads();
        if (tid == 0) {
            const int64_t blin = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            for (int k = 0; k < 7; ++k) {
                double t = 0.0;
                for (int wv = 0; wv < (NT + 63) / 64; ++wv) t += red[wv][k];
                s.diag_partial[blin * kDiag + k] = t;
            }
            s.diag_partial[blin * kDiag + 7] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers

template <int BX, int BY, typename TIN, typename TOUT, typename CT>
static hipError_t launch_t(const Consts &c, const StageArgs &s, hipStream_t st)
{
    dim3 block(BX, BY, 1);
    dim3 grid((c.nx + BX - 1) / BX, (c.ny + BY - 1) / BY, (c.nz + s.zchunk - 1) / s.zchunk);
    hipLaunchKernelGGL((fused_stage_kernel<BX, BY, TIN, TOUT, CT>), grid, block, 0, st, c, s);
    return hipGetLastError();
}

template <typename TIN, typename TOUT, typename CT>
static hipError_t launch_tile(int tile, const Consts &c, const StageArgs &s, hipStream_t st)
{
    switch (tile) {
    case TILE_32x8: return launch_t<32, 8, TIN, TOUT, CT>(c, s, st);
    case TILE_16x16: return launch_t<16, 16, TIN, TOUT, CT>(c, s, st);
    case TILE_64x4: return launch_t<64, 4, TIN, TOUT, CT>(c, s, st);
    case TILE_32x16: return launch_t<32, 16, TIN, TOUT, CT>(c, s, st);
    default: return hipErrorInvalidValue;
    }
}

void tile_dims(int tile, int *bx, int *by)
{
    switch (tile) {
    case TILE_16x16: *bx = 16; *by = 16; break;
    case TILE_64x4: *bx = 64; *by = 4; break;
    case TILE_32x16: *bx = 32; *by = 16; break;
    default: *bx = 32; *by = 8; break;
    }
}

int64_t fused_num_blocks(const Consts &c, int tile, int zchunk)
{
    int bx, by;
    tile_dims(tile, &bx, &by);
    return (int64_t)((c.nx + bx - 1) / bx) * ((c.ny + by - 1) / by) * ((c.nz + zchunk - 1) / zchunk);
}

hipError_t launch_fused_stage(const Consts &c, const StageArgs &s, ns_precision prec,
                              int tile, hipStream_t st)
{
    if (prec == NS_FP64)
        return launch_tile<double, double, double>(tile, c, s, st);
    // FP32 storage: stage 1 reads the double state, stage 3 writes it.
    if (s.mode == 1) return launch_tile<double, float, float>(tile, c, s, st);
    if (s.mode == 2) return launch_tile<float, float, float>(tile, c, s, st);
    return launch_tile<float, double, float>(tile, c, s, st);
}

}  // namespace ns
