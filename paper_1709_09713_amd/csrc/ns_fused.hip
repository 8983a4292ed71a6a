// ns_fused.hip -- the fused on-the-fly residual + RK3 stage kernel.
//
// This is the minimal-storage algorithm class of the algorithms section
// (RA / SN / SN2): no derivative is written to a global array.  Every
// derivative of the mass, momentum and energy equations (methodology
// section; stencils fd and sd) is evaluated on the fly and accumulated
// straight into the residual registers of its grid point, and the
// low-storage RK3 update of the generic-algorithm figure is applied in the
// same pass, so a stage reads its input once and writes its outputs once.
//
// MI355X mapping:
//  * A block owns a BX x BY column tile of the (x, y) plane and marches
//    along z through a chunk of planes.  Each plane of the tile plus a
//    radius-2 halo (wrap-around indexing replaces the periodic-boundary
//    pass) is loaded with coalesced x-fastest loads one plane ahead of its
//    use (software prefetch into registers), turned into the primitive
//    variables once per point, and staged in LDS (double buffered, one
//    barrier per plane).  x and y stencil taps are LDS reads.
//  * z derivatives whose coefficient is a constant (the flux divergences
//    d(rho w)/dz, d(rho u_i w)/dz, dp/dz, d((rho E/2 + p) w)/dz and the heat
//    conduction d2T/dz2) are scattered: as soon as a plane is staged its
//    values are added, with the stencil weights, into a five-deep ring of
//    pending residual accumulators of the planes two below to two above it
//    (linearity lets terms that share a coefficient share one stencil).
//  * z derivatives multiplied by point values (w d(rho, rho u_i, rho E)/dz,
//    the velocity gradient, the viscous terms) are gathered at the output
//    plane from a five-deep register ring of (rho, rho E, u, v, w).
//  * Mixed derivatives that involve z are taken as z-derivatives of in-plane
//    derivatives (D_x D_z w = D_z D_x w, exact in exact arithmetic), so
//    three in-plane quantities (D_x u + D_y v, D_x w, D_y w) get a ring;
//    D_x D_y is a 16-tap LDS stencil.
//  * The march is unrolled by the ring depth (5) so every ring slot is a
//    compile-time register: no rotation moves.
//  * Stage 1 can also emit per-block partial sums of the diagnostics of its
//    input state, so the per-step diagnostics cost no extra pass.
//
// Precision: CT is the stencil/residual arithmetic type.  With CT = float
// (FP32 storage) the staged fields are deviations from the uniform
// reference state (rho - 1, rhoE - rhoE_ref, p - p_ref, T - 1); the constant
// parts are applied analytically (stencil coefficients sum to zero: only
// H_ref div u survives, added in double), and the RK accumulator stays
// double.
#include <atomic>
#include <type_traits>

#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

template <typename TIN, typename CT>
__device__ __forceinline__ CT to_ct(TIN v, double ref)
{
    if constexpr (std::is_same<CT, double>::value)
        return v;
    else if constexpr (std::is_same<TIN, double>::value)
        return (float)(v - ref);
    else
        return v;
}

// Stage outputs and the accumulator are streamed: written (or read) once
// per stage and not touched again before the next stage, which rereads them
// from HBM anyway.  Non-temporal accesses keep them from displacing the
// input planes in L2, whose halo rows neighbouring blocks read again.
template <typename TOUT>
__device__ __forceinline__ void store_q(void *q, int64_t i, double v, double ref)
{
    if constexpr (std::is_same<TOUT, double>::value)
        __builtin_nontemporal_store(v, (double *)q + i);
    else
        __builtin_nontemporal_store((float)(v - ref), (float *)q + i);
}

template <int V>
using IC = std::integral_constant<int, V>;

// 1/x from the hardware reciprocal estimate refined by Newton steps
// (r <- r + r (1 - x r)): two steps reach double rounding error, one step
// single.  Cheaper than the IEEE division sequence; the density is
// positive and far from the denormal range.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// ORD selects the evaluation order of the in-plane residual terms (the
// SN / SN2 distinction of the minimal-storage section): 0 groups them by
// equation, the momentum equations by velocity component; 1 groups them by
// derivative direction.  Same terms, different association of the sums.
//
// PAIR (even nx; not with the FP32 stage-1 own-column loads): each load
// slot covers two x-neighbours with one 2-wide load.  Pairs start at even x,
// so with nx even they never straddle the periodic wrap.
template <int BX, int BY, typename TIN, typename TOUT, typename CT, bool DIAG, int ORD, bool PAIR>
__global__ void __launch_bounds__(BX * BY)
fused_stage_kernel(Consts c, StageArgs s)
{
    // Multiply-adds are fused only within one expression: the five unrolled
    // phases of the march then round alike, so a point's result does not
    // depend on where its plane falls in a z-chunk.
#pragma clang fp contract(on)
    constexpr bool DEV = std::is_same<CT, float>::value;
    static_assert(BX % 2 == 0, "pairs need an even tile width");
    static_assert(!(PAIR && DEV && std::is_same<TIN, double>::value), "own-column loads are single");
    constexpr int HX = BX + 4, HY = BY + 4, HP = HX * HY, NT = BX * BY;
    constexpr int PW = PAIR ? 2 : 1;                       // points per load slot
    constexpr int NLOAD = (HP + PW * NT - 1) / (PW * NT);
    enum { L_RHO, L_M0, L_M1, L_M2, L_E, L_U, L_V, L_W, L_P, L_T, NF };
    enum { Z_RHO, Z_E, Z_U, Z_V, Z_W, NZ };
    static_assert(HP % 2 == 0, "pair cells start at even LDS offsets");
    __shared__ __attribute__((aligned(16))) CT lds[2][NF][HP];
    __shared__ double red[NT / 64 + 1][kDiag];

    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    int tbx, tby, tbz;
    xcd_tile(&tbx, &tby, &tbz);
    const int x0 = tbx * BX, y0 = tby * BY;
    const int z0 = tbz * s.zchunk;
    const int z1 = min(z0 + s.zchunk, c.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = (gx < c.nx) && (gy < c.ny);
    const int own = (ty + 2) * HX + tx + 2;
    const int64_t N = c.N;
    const TIN *qin = (const TIN *)s.qin;
    constexpr int NR = DIAG ? 6 : 5;    // ring entries: residuals (+ omega_z)
    const int64_t col = (int64_t)gy * c.nx + gx;   // own (x, y) offset in a plane

    // FP32 storage, stage 1: the input is the exact double state, which is
    // also the RK accumulator of the output point.  Each thread then loads
    // its own column as load slot 0 (the halo ring goes to the other slots)
    // and keeps that point's doubles for the three steps until the point is
    // finished, instead of reading them from memory a second time.
    constexpr bool OWN = DEV && std::is_same<TIN, double>::value;

    // Plane offsets and LDS cells of the points this thread loads (fixed
    // for the march); lcell < 0 marks an unused slot.
    int loff[NLOAD], lcell[NLOAD];
#pragma unroll
    for (int r = 0; r < NLOAD; ++r) {
        int lx = 0, ly = 0;
        lcell[r] = -1;
        if constexpr (OWN) {
            if (r == 0) {
                lx = tx + 2;
                ly = ty + 2;
                lcell[r] = ly * HX + lx;
            } else {
                // k-th point of the radius-2 ring around the tile: two rows
                // on top, two at the bottom, then two columns on each side
                const int k = tid + (r - 1) * NT;
                if (k < HP - NT) {
                    if (k < 4 * HX) {
                        const int row = k / HX;
                        lx = k % HX;
                        ly = row < 2 ? row : HY - 4 + row;
                    } else {
                        const int q = k - 4 * HX, cc = q % 4;
                        ly = 2 + q / 4;
                        lx = cc < 2 ? cc : HX - 4 + cc;
                    }
                    lcell[r] = ly * HX + lx;
                }
            }
        } else if constexpr (PAIR) {
            const int q = tid + r * NT;            // pair index
            if (q < HP / 2) {
                lx = 2 * (q % (HX / 2));
                ly = q / (HX / 2);
                lcell[r] = ly * HX + lx;
            }
        } else {
            const int idx = tid + r * NT;
            if (idx < HP) {
                lx = idx % HX;
                ly = idx / HX;
                lcell[r] = idx;
            }
        }
        loff[r] = 0;
        if (lcell[r] >= 0) {
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
    const CT kz = kappa * c2z;

    CT qz[5][NZ];                 // ring: (rho, rhoE, u, v, w) of the own column
    CT qa[5], qb[5], qc[5];       // ring: D_x u + D_y v, D_x w, D_y w
    CT ra[5][NR];                 // ring: pending residuals (5) (+ omega_z)
    // Vector memory counters retire loads and stores in issue order, so a
    // wait for a load issued after a store also waits for that store.  With
    // FP32 storage (stages 2 and 3, and the residual) the next plane is
    // therefore loaded two steps ahead (pg, copied into pf at the end of a
    // step) and the accumulator of the next step's output point one step
    // ahead, both before the step's stores.  FP64 storage, whose doubled
    // prefetch registers cost more than the ordering gains (measured), and
    // the own-column stage 1 of FP32 storage, short of registers, load one
    // plane ahead and the accumulator at the start of its step.
    constexpr bool AHEAD2 = !OWN && std::is_same<TIN, float>::value;
    TIN pf[NLOAD][5][PW];         // plane zp + 1, staged in step zp
    TIN pg[AHEAD2 ? NLOAD : 1][5][PW];   // plane zp + 2, loaded in step zp (AHEAD2)
    double accpf[5];              // accumulator (or exact state) of the output point
    double accn[5];               // the next step's, prefetched (AHEAD2)
    double ocol[3][5];            // exact state of the own column, three planes (OWN only)
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int f = 0; f < 5; ++f) ocol[q][f] = 0.0;
#pragma unroll
    for (int f = 0; f < 5; ++f) accpf[f] = accn[f] = 0.0;
    double dsum[DIAG ? 7 : 1];
#pragma unroll
    for (int k = 0; k < (DIAG ? 7 : 1); ++k) dsum[k] = 0.0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        qa[q] = qb[q] = qc[q] = CT(0);
#pragma unroll
        for (int f = 0; f < NZ; ++f) qz[q][f] = CT(0);
#pragma unroll
        for (int f = 0; f < NR; ++f) ra[q][f] = CT(0);
    }

    auto load_plane = [&](int zp, TIN (&dst)[NLOAD][5][PW]) {
        // zp is in [-2, nz + 6] (march padding): at most two wraps
        int zw = zp < 0 ? zp + c.nz : zp;
        zw = zw >= c.nz ? zw - c.nz : zw;
        zw = zw >= c.nz ? zw - c.nz : zw;
        const int64_t base = (int64_t)zw * c.nxy;
        // every slot loads (idle slots read a valid point they never use):
        // unconditional loads keep the wait counts exact
#pragma unroll
        for (int r = 0; r < NLOAD; ++r) {
            const int64_t g = base + loff[r];
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                if constexpr (PAIR) {
                    typedef TIN pair_t __attribute__((ext_vector_type(2)));
                    const pair_t v = *(const pair_t *)(qin + g + f * N);
                    dst[r][f][0] = v.x;
                    dst[r][f][1] = v.y;
                } else {
                    dst[r][f][0] = qin[g + f * N];
                }
            }
        }
    };
    // conserved (pf) -> primitives -> LDS buffer b
    auto stage_plane = [&](int b) {
#pragma unroll
        for (int r = 0; r < NLOAD; ++r) {
            if (lcell[r] < 0) continue;
            CT val[NF][PW];
#pragma unroll
            for (int j = 0; j < PW; ++j) {
                const CT rho = to_ct<TIN, CT>(pf[r][0][j], c.rho_ref);
                const CT m0 = to_ct<TIN, CT>(pf[r][1][j], 0.0);
                const CT m1 = to_ct<TIN, CT>(pf[r][2][j], 0.0);
                const CT m2 = to_ct<TIN, CT>(pf[r][3][j], 0.0);
                const CT E = to_ct<TIN, CT>(pf[r][4][j], c.rhoE_ref);
                const CT rhof = DEV ? CT(1) + rho : rho;
                const CT inv = recip(rhof);
                const CT u = m0 * inv, v = m1 * inv, w = m2 * inv;
                const CT p = gm1 * (E - half * (m0 * u + m1 * v + m2 * w));
                // T = gamma M^2 p / rho; as a deviation from T = 1 when the
                // reference state satisfies gamma M^2 p_ref = rho_ref = 1.
                const CT T = DEV ? (gM2 * p - rho) * inv : gM2 * p * inv;
                val[L_RHO][j] = rho;
                val[L_M0][j] = m0;
                val[L_M1][j] = m1;
                val[L_M2][j] = m2;
                val[L_E][j] = E;
                val[L_U][j] = u;
                val[L_V][j] = v;
                val[L_W][j] = w;
                val[L_P][j] = p;
                val[L_T][j] = T;
            }
            const int idx = lcell[r];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if constexpr (PAIR) {
                    // one 2-wide LDS store per field and pair (idx is even)
                    typedef CT pair_t __attribute__((ext_vector_type(2)));
                    pair_t v2;
                    v2.x = val[f][0];
                    v2.y = val[f][1];
                    ((pair_t *)&lds[b][f][0])[idx >> 1] = v2;
                } else {
                    lds[b][f][idx] = val[f][0];
                }
            }
        }
    };

    // own-column ring: planes zp+1, zp, zp-1 after the shift at the end of step zp
    auto shift_ocol = [&]() {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            ocol[2][f] = ocol[1][f];
            ocol[1][f] = ocol[0][f];
            ocol[0][f] = (double)pf[0][f][0];
        }
    };

    // One plane of the march.  PH = (zp - z0 + 2) mod 5 selects ring slots:
    // plane zp + k lives in slot (PH + k) mod 5.
    auto step = [&](auto phc, int zp) {
        constexpr int PH = decltype(phc)::value;
        constexpr int SM2 = (PH + 3) % 5, SM1 = (PH + 4) % 5, S0 = PH;
        constexpr int SP1 = (PH + 1) % 5, SP2 = (PH + 2) % 5;
        constexpr int SM4 = (PH + 1) % 5, SM3 = (PH + 2) % 5;   // zp-4, zp-3
        const int b = (zp - z0) & 1;
        const int zf = zp - 2;
        const bool fin = active && zf >= z0 && zf < z1;

        // issue the loads of the next planes and accumulators (see above);
        // threads with no output point read a valid address they ignore
        // stages 2 and 3 read the accumulator; the residual and stage 1
        // read the exact double input state (unused for the residual)
        const double *src = (s.mode >= 2) ? s.acc_in : (const double *)s.qin;
        if constexpr (AHEAD2) {
            load_plane(zp + 2, pg);
            const int zn = zf + 1;
            const int64_t pn = (int64_t)((active && zn >= z0 && zn < z1) ? zn : z0) * c.nxy
                               + (active ? col : 0);
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                accpf[f] = accn[f];
                accn[f] = __builtin_nontemporal_load(src + f * N + pn);
            }
        } else if constexpr (OWN) {
            // stage 1 of FP32 storage: the exact state of plane zp - 2,
            // loaded three steps ago as this thread's slot 0
#pragma unroll
            for (int f = 0; f < 5; ++f) accpf[f] = ocol[2][f];
            load_plane(zp + 1, pf);
        } else {
            // the accumulator, needed first, is requested first
            const int64_t pidx = (int64_t)(fin ? zf : z0) * c.nxy + (active ? col : 0);
#pragma unroll
            for (int f = 0; f < 5; ++f) accpf[f] = __builtin_nontemporal_load(src + f * N + pidx);
            load_plane(zp + 1, pf);
        }

        // the slot of plane zp + 2 is free (plane zp - 3 was finished)
#pragma unroll
        for (int f = 0; f < NR; ++f) ra[SP2][f] = CT(0);

#define LV(f, dy, dx) lds[b][f][own + (dy) * HX + (dx)]
#define DX1(f) d1u(LV(f, 0, -2), LV(f, 0, -1), LV(f, 0, 1), LV(f, 0, 2))
#define DY1(f) d1u(LV(f, -2, 0), LV(f, -1, 0), LV(f, 1, 0), LV(f, 2, 0))
#define DX1P(f, g)                                                       \
    d1u(LV(f, 0, -2) * LV(g, 0, -2), LV(f, 0, -1) * LV(g, 0, -1),        \
        LV(f, 0, 1) * LV(g, 0, 1), LV(f, 0, 2) * LV(g, 0, 2))
#define DY1P(f, g)                                                       \
    d1u(LV(f, -2, 0) * LV(g, -2, 0), LV(f, -1, 0) * LV(g, -1, 0),        \
        LV(f, 1, 0) * LV(g, 1, 0), LV(f, 2, 0) * LV(g, 2, 0))
// (rhoE/2 + p) u_j at a tap: energy flux of the x or y direction
#define HF(dy, dx, g) ((half * LV(L_E, dy, dx) + LV(L_P, dy, dx)) * LV(g, dy, dx))
#define DX1H() d1u(HF(0, -2, L_U), HF(0, -1, L_U), HF(0, 1, L_U), HF(0, 2, L_U))
#define DY1H() d1u(HF(-2, 0, L_V), HF(-1, 0, L_V), HF(1, 0, L_V), HF(2, 0, L_V))
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

        if (active) {
            const CT rho = LV(L_RHO, 0, 0), E = LV(L_E, 0, 0);
            const CT m0 = LV(L_M0, 0, 0), m1 = LV(L_M1, 0, 0), m2 = LV(L_M2, 0, 0);
            const CT u = LV(L_U, 0, 0), v = LV(L_V, 0, 0), w = LV(L_W, 0, 0);
            const CT p = LV(L_P, 0, 0), T = LV(L_T, 0, 0);
            const CT Gxx = c1x * DX1(L_U), Gxy = c1y * DY1(L_U);
            const CT Gyx = c1x * DX1(L_V), Gyy = c1y * DY1(L_V);
            const CT Gzx = c1x * DX1(L_W), Gzy = c1y * DY1(L_W);
            const CT a = Gxx + Gyy;
            qz[S0][Z_RHO] = rho;
            qz[S0][Z_E] = E;
            qz[S0][Z_U] = u;
            qz[S0][Z_V] = v;
            qz[S0][Z_W] = w;
            qa[S0] = a;
            qb[S0] = Gzx;
            qc[S0] = Gzy;

            // scatter the constant-coefficient z fluxes of this plane
            const CT g0 = -half * c1z * m2;                  // -1/2 d(rho w)/dz
            const CT g1 = -half * c1z * (m0 * w);            // -1/2 d(rho u w)/dz
            const CT g2 = -half * c1z * (m1 * w);            // -1/2 d(rho v w)/dz
            const CT g3 = -c1z * (half * (m2 * w) + p);      // -1/2 d(rho w w)/dz - dp/dz
            const CT g4 = -c1z * ((half * E + p) * w);       // -1/2 d(rhoE w)/dz - d(p w)/dz
            const CT gT = kz * T;                            // kappa d2T/dz2
            const CT g[5] = {g0, g1, g2, g3, g4};
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                ra[SM2][f] -= g[f];
                ra[SM1][f] += CT(8) * g[f];
                ra[SP1][f] -= CT(8) * g[f];
                ra[SP2][f] += g[f];
            }
            ra[SM2][4] -= gT;
            ra[SM1][4] += CT(16) * gT;
            ra[S0][4] -= CT(30) * gT;
            ra[SP1][4] += CT(16) * gT;
            ra[SP2][4] -= gT;

            if (zp >= z0 && zp < z1) {
                // in-plane (x, y) part of the residual of this plane
                const CT rhof = DEV ? CT(1) + rho : rho;
                const CT uc = u * c1x, vc = v * c1y;
                // tau_ij du_i/dx_j restricted to terms without a z derivative
                auto in_plane_phi = [&]() {
                    return CT(2) * (Gxx * Gxx + Gyy * Gyy) + Gxy * Gxy + Gyx * Gyx
                           + CT(2) * Gxy * Gyx + Gzx * Gzx + Gzy * Gzy;
                };
                if constexpr (ORD == 0) {
                    // grouped by equation (momentum by velocity component)
                    ra[S0][0] -= half * (c1x * DX1(L_M0) + c1y * DY1(L_M1) + rhof * a
                                         + uc * DX1(L_RHO) + vc * DY1(L_RHO));
                    ra[S0][1] -= half * (c1x * DX1P(L_M0, L_U) + c1y * DY1P(L_M0, L_V) + m0 * a
                                         + uc * DX1(L_M0) + vc * DY1(L_M0))
                                 + c1x * DX1(L_P);
                    ra[S0][2] -= half * (c1x * DX1P(L_M1, L_U) + c1y * DY1P(L_M1, L_V) + m1 * a
                                         + uc * DX1(L_M1) + vc * DY1(L_M1))
                                 + c1y * DY1(L_P);
                    ra[S0][3] -= half * (c1x * DX1P(L_M2, L_U) + c1y * DY1P(L_M2, L_V) + m2 * a
                                         + uc * DX1(L_M2) + vc * DY1(L_M2));
                    // viscous: d_j tau_ij = lap u_i + (1/3) d_i div u, in-plane parts
                    const CT Vx = four3 * (c2x * DX2(L_U)) + c2y * DY2(L_U)
                                  + third * (c1x * c1y * DXDY(L_V));
                    const CT Vy = c2x * DX2(L_V) + four3 * (c2y * DY2(L_V))
                                  + third * (c1x * c1y * DYDX(L_U));
                    const CT Vz = c2x * DX2(L_W) + c2y * DY2(L_W);
                    ra[S0][1] += inv_re * Vx;
                    ra[S0][2] += inv_re * Vy;
                    ra[S0][3] += inv_re * Vz;
                    const CT phi = in_plane_phi();
                    // energy: skew convection, pressure work, viscous work,
                    // dissipation, heat conduction (x, y)
                    ra[S0][4] += -(c1x * DX1H() + c1y * DY1H())
                                 - half * (E * a + uc * DX1(L_E) + vc * DY1(L_E))
                                 + inv_re * (u * Vx + v * Vy + w * Vz + phi)
                                 + kappa * (c2x * DX2(L_T) + c2y * DY2(L_T));
                } else {
                    // grouped by direction: every x derivative of every
                    // equation, then every y derivative
                    const CT phi = in_plane_phi();
                    CT r0 = rhof * a, r1 = m0 * a, r2 = m1 * a, r3 = m2 * a, r4 = E * a;
                    CT Vx = third * (c1x * c1y * DXDY(L_V));
                    CT Vy = third * (c1x * c1y * DYDX(L_U));
                    r0 += c1x * DX1(L_M0) + uc * DX1(L_RHO);
                    r1 += c1x * DX1P(L_M0, L_U) + uc * DX1(L_M0);
                    r2 += c1x * DX1P(L_M1, L_U) + uc * DX1(L_M1);
                    r3 += c1x * DX1P(L_M2, L_U) + uc * DX1(L_M2);
                    r4 += uc * DX1(L_E);
                    CT h = c1x * DX1H();
                    const CT px = c1x * DX1(L_P);
                    Vx += four3 * (c2x * DX2(L_U));
                    Vy += c2x * DX2(L_V);
                    CT Vz = c2x * DX2(L_W);
                    CT lapT = c2x * DX2(L_T);
                    r0 += c1y * DY1(L_M1) + vc * DY1(L_RHO);
                    r1 += c1y * DY1P(L_M0, L_V) + vc * DY1(L_M0);
                    r2 += c1y * DY1P(L_M1, L_V) + vc * DY1(L_M1);
                    r3 += c1y * DY1P(L_M2, L_V) + vc * DY1(L_M2);
                    r4 += vc * DY1(L_E);
                    h += c1y * DY1H();
                    const CT py = c1y * DY1(L_P);
                    Vx += c2y * DY2(L_U);
                    Vy += four3 * (c2y * DY2(L_V));
                    Vz += c2y * DY2(L_W);
                    lapT += c2y * DY2(L_T);
                    ra[S0][0] -= half * r0;
                    ra[S0][1] += inv_re * Vx - (half * r1 + px);
                    ra[S0][2] += inv_re * Vy - (half * r2 + py);
                    ra[S0][3] += inv_re * Vz - half * r3;
                    ra[S0][4] += -h - half * r4 + inv_re * (u * Vx + v * Vy + w * Vz + phi)
                                 + kappa * lapT;
                }
                if constexpr (DIAG) ra[S0][NR - 1] = Gyx - Gxy;   // omega_z
            }
        }
#undef LV
#undef DX1
#undef DY1
#undef DX1P
#undef DY1P
#undef HF
#undef DX1H
#undef DY1H
#undef DX2
#undef DY2
#undef DXDY
#undef DYDX

        // ---- stage plane zp + 1 into the other LDS buffer (last read in the
        // previous step, before its barrier); done before the output stores
        // so that waiting for the prefetched loads never waits for stores
        stage_plane(b ^ 1);

        // ---- finish plane zf = zp - 2: gathered z terms, RK update, output
        if (fin) {
#define DZ1(f) d1u(qz[SM4][f], qz[SM3][f], qz[SM1][f], qz[S0][f])
#define DZ2(f) d2u(qz[SM4][f], qz[SM3][f], qz[SM2][f], qz[SM1][f], qz[S0][f])
#define DZM(k)                                                                       \
    d1u(qz[SM4][Z_RHO] * qz[SM4][k], qz[SM3][Z_RHO] * qz[SM3][k],                    \
        qz[SM1][Z_RHO] * qz[SM1][k], qz[S0][Z_RHO] * qz[S0][k])
            const CT rho = qz[SM2][Z_RHO], E = qz[SM2][Z_E];
            const CT u = qz[SM2][Z_U], v = qz[SM2][Z_V], w = qz[SM2][Z_W];
            const CT rhof = DEV ? CT(1) + rho : rho;
            const CT a = qa[SM2], bb = qb[SM2], cc = qc[SM2];
            const CT wc = w * c1z;
            const CT Gxz = c1z * DZ1(Z_U), Gyz = c1z * DZ1(Z_V), Gzz = c1z * DZ1(Z_W);
            const CT Da = c1z * d1u(qa[SM4], qa[SM3], qa[SM1], qa[S0]);
            const CT Db = c1z * d1u(qb[SM4], qb[SM3], qb[SM1], qb[S0]);
            const CT Dc = c1z * d1u(qc[SM4], qc[SM3], qc[SM1], qc[S0]);
            // rho u_i at the z taps (m_i = rho u_i; in the deviation form
            // rho is 1 + rho')
            CT R[5];
            R[0] = ra[SM2][0] - half * (rhof * Gzz + wc * DZ1(Z_RHO));
            if constexpr (DEV) {
#define DZMD(k)                                                                                    \
    d1u((CT(1) + qz[SM4][Z_RHO]) * qz[SM4][k], (CT(1) + qz[SM3][Z_RHO]) * qz[SM3][k],              \
        (CT(1) + qz[SM1][Z_RHO]) * qz[SM1][k], (CT(1) + qz[S0][Z_RHO]) * qz[S0][k])
                R[1] = ra[SM2][1] - half * (rhof * u * Gzz + wc * DZMD(Z_U));
                R[2] = ra[SM2][2] - half * (rhof * v * Gzz + wc * DZMD(Z_V));
                R[3] = ra[SM2][3] - half * (rhof * w * Gzz + wc * DZMD(Z_W));
#undef DZMD
            } else {
                R[1] = ra[SM2][1] - half * (rhof * u * Gzz + wc * DZM(Z_U));
                R[2] = ra[SM2][2] - half * (rhof * v * Gzz + wc * DZM(Z_V));
                R[3] = ra[SM2][3] - half * (rhof * w * Gzz + wc * DZM(Z_W));
            }
            const CT Vx = c2z * DZ2(Z_U) + third * Db;
            const CT Vy = c2z * DZ2(Z_V) + third * Dc;
            const CT Vz = four3 * (c2z * DZ2(Z_W)) + third * Da;
            R[1] += inv_re * Vx;
            R[2] += inv_re * Vy;
            R[3] += inv_re * Vz;
            const CT div = a + Gzz;
            const CT phi = Gxz * Gxz + Gyz * Gyz + CT(2) * Gzz * Gzz
                           + CT(2) * (Gxz * bb + Gyz * cc) - two3 * div * div;
            R[4] = ra[SM2][4] - half * (E * Gzz + wc * DZ1(Z_E))
                   + inv_re * (u * Vx + v * Vy + w * Vz + phi);
#undef DZ1
#undef DZ2
#undef DZM
            double Rd[5];
#pragma unroll
            for (int f = 0; f < 5; ++f) Rd[f] = (double)R[f];
            if constexpr (DEV) Rd[4] -= c.H_ref * ((double)a + (double)Gzz);

            const int64_t pidx = (int64_t)zf * c.nxy + col;
            if (s.mode == 0) {
#pragma unroll
                for (int f = 0; f < 5; ++f) s.rout[f * N + pidx] = Rd[f];
            } else {
                const double ref[5] = {c.rho_ref, 0.0, 0.0, 0.0, c.rhoE_ref};
                if constexpr (DIAG) {
                    // diagnostics of the stage input (the state at step
                    // start): conserved totals from the exact double state,
                    // kinetic energy and enstrophy from the staged
                    // primitives and gradients
                    const CT ox = cc - Gyz, oy = Gxz - bb, oz = ra[SM2][NR - 1];
#pragma unroll
                    for (int f = 0; f < 5; ++f) dsum[f] += accpf[f];
                    dsum[5] += 0.5 * (accpf[1] * (double)u + accpf[2] * (double)v
                                      + accpf[3] * (double)w);
                    dsum[6] += 0.5 * (double)rhof * ((double)ox * (double)ox + (double)oy * (double)oy
                                                     + (double)oz * (double)oz);
                }
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    store_q<TOUT>(s.qout, f * N + pidx, accpf[f] + s.a_dt * Rd[f], ref[f]);
                    if (s.mode < 3)
                        __builtin_nontemporal_store(accpf[f] + s.b_dt * Rd[f], s.acc_out + f * N + pidx);
                }
            }
        }

        if constexpr (OWN) shift_ocol();
        if constexpr (AHEAD2) {
#pragma unroll
            for (int r = 0; r < NLOAD; ++r)
#pragma unroll
                for (int f = 0; f < 5; ++f)
#pragma unroll
                    for (int j = 0; j < PW; ++j) pf[r][f][j] = pg[r][f][j];
        }
        lds_barrier();
    };

    // prologue: plane z0 - 2 into LDS buffer 0
    load_plane(z0 - 2, pf);
    stage_plane(0);
    if constexpr (OWN) shift_ocol();
    if constexpr (AHEAD2) load_plane(z0 - 1, pf);
    lds_barrier();

    // The march covers planes z0-2 .. z1+1, padded to a multiple of 5;
    // padding planes are loaded (wrapped, valid memory) but never output.
    const int L = z1 - z0 + 4;
    for (int it = 0; it < L; it += 5) {
        const int zp = z0 - 2 + it;
        step(IC<0>{}, zp);
        step(IC<1>{}, zp + 1);
        step(IC<2>{}, zp + 2);
        step(IC<3>{}, zp + 3);
        step(IC<4>{}, zp + 4);
    }

    if constexpr (DIAG) {
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

template <int BX, int BY, typename TIN, typename TOUT, typename CT, int ORD>
static hipError_t launch_o(const Consts &c, const StageArgs &s, hipStream_t st)
{
    dim3 block(BX, BY, 1);
    dim3 grid((c.nx + BX - 1) / BX, (c.ny + BY - 1) / BY, (c.nz + s.zchunk - 1) / s.zchunk);
    // per-step diagnostics are only taken in stage 1, which reads the
    // double state
    // paired plane loads need an even x extent; the FP32 stage-1 kernel
    // loads single points (own-column accumulator)
    constexpr bool CAN_PAIR = !(std::is_same<CT, float>::value && std::is_same<TIN, double>::value);
    const bool pair = CAN_PAIR && c.nx % 2 == 0;
    if constexpr (std::is_same<TIN, double>::value) {
        if (s.diag_partial != nullptr && s.mode == 1) {
            if (pair)
                hipLaunchKernelGGL((fused_stage_kernel<BX, BY, TIN, TOUT, CT, true, ORD, CAN_PAIR>), grid,
                                   block, 0, st, c, s);
            else
                hipLaunchKernelGGL((fused_stage_kernel<BX, BY, TIN, TOUT, CT, true, ORD, false>), grid, block,
                                   0, st, c, s);
            return hipGetLastError();
        }
    }
    if (pair)
        hipLaunchKernelGGL((fused_stage_kernel<BX, BY, TIN, TOUT, CT, false, ORD, CAN_PAIR>), grid, block, 0,
                           st, c, s);
    else
        hipLaunchKernelGGL((fused_stage_kernel<BX, BY, TIN, TOUT, CT, false, ORD, false>), grid, block, 0, st,
                           c, s);
    return hipGetLastError();
}

// The direction-grouped order is compiled for the default tile of each
// precision only (16x8 and 32x8); order_supported() tells the host.
template <int BX, int BY, typename TIN, typename TOUT, typename CT>
static hipError_t launch_t(const Consts &c, const StageArgs &s, hipStream_t st)
{
    if (s.order == 0) return launch_o<BX, BY, TIN, TOUT, CT, 0>(c, s, st);
    if constexpr ((BX == 16 && BY == 8) || (BX == 32 && BY == 8))
        return launch_o<BX, BY, TIN, TOUT, CT, 1>(c, s, st);
    return hipErrorInvalidValue;
}

template <typename TIN, typename TOUT, typename CT>
static hipError_t launch_tile(int tile, const Consts &c, const StageArgs &s, hipStream_t st)
{
    switch (tile) {
    case TILE_32x8: return launch_t<32, 8, TIN, TOUT, CT>(c, s, st);
    case TILE_16x16: return launch_t<16, 16, TIN, TOUT, CT>(c, s, st);
    case TILE_64x4: return launch_t<64, 4, TIN, TOUT, CT>(c, s, st);
    case TILE_32x16: return launch_t<32, 16, TIN, TOUT, CT>(c, s, st);
    case TILE_16x8: return launch_t<16, 8, TIN, TOUT, CT>(c, s, st);
    case TILE_32x4: return launch_t<32, 4, TIN, TOUT, CT>(c, s, st);
    case TILE_16x4: return launch_t<16, 4, TIN, TOUT, CT>(c, s, st);
    case TILE_8x8: return launch_t<8, 8, TIN, TOUT, CT>(c, s, st);
    default: return hipErrorInvalidValue;
    }
}

void tile_dims(int tile, int *bx, int *by)
{
    switch (tile) {
    case TILE_16x16: *bx = 16; *by = 16; break;
    case TILE_64x4: *bx = 64; *by = 4; break;
    case TILE_32x16: *bx = 32; *by = 16; break;
    case TILE_16x8: *bx = 16; *by = 8; break;
    case TILE_32x4: *bx = 32; *by = 4; break;
    case TILE_16x4: *bx = 16; *by = 4; break;
    case TILE_8x8: *bx = 8; *by = 8; break;
    case TILE_16x8_2G: *bx = 16; *by = 8; break;
    case TILE_16x4_2G: *bx = 16; *by = 4; break;
    default: *bx = 32; *by = 8; break;
    }
}

// Blocks of one stage kernel instance that the device holds at once
// (compute units x occupancy per compute unit); 0 if it cannot be queried.
template <int BX, int BY, typename TIN, typename TOUT, typename CT>
static int resident_t()
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(&fused_stage_kernel<BX, BY, TIN, TOUT, CT, false, 0, false>),
            BX * BY, 0) != hipSuccess)
        return 0;
    return cus * (per > 0 ? per : 1);
}

template <typename TIN, typename TOUT, typename CT>
static int resident_tile(int tile)
{
    switch (tile) {
    case TILE_32x8: return resident_t<32, 8, TIN, TOUT, CT>();
    case TILE_16x16: return resident_t<16, 16, TIN, TOUT, CT>();
    case TILE_64x4: return resident_t<64, 4, TIN, TOUT, CT>();
    case TILE_32x16: return resident_t<32, 16, TIN, TOUT, CT>();
    case TILE_16x8: return resident_t<16, 8, TIN, TOUT, CT>();
    case TILE_32x4: return resident_t<32, 4, TIN, TOUT, CT>();
    case TILE_16x4: return resident_t<16, 4, TIN, TOUT, CT>();
    case TILE_8x8: return resident_t<8, 8, TIN, TOUT, CT>();
    default: return 0;
    }
}

int fused_resident_blocks(ns_precision prec, int tile)
{
    if (tile < 0 || tile >= TILE_COUNT) return 0;
    // queried once per (device, precision, tile)
    constexpr int kMaxDev = 16;
    static std::atomic<int> cache[kMaxDev][2][TILE_COUNT];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0;
    const int q = prec == NS_FP64 ? 0 : 1;
    int r = cache[dev][q][tile].load();
    if (r == 0) {
        if (split_tile(tile))
            r = split_resident_blocks(prec, tile);
        else
            r = prec == NS_FP64 ? resident_tile<double, double, double>(tile)
                                : resident_tile<float, float, float>(tile);
        if (r > 0) cache[dev][q][tile].store(r);
    }
    return r;
}

bool fused_order_supported(int tile, int order)
{
    return order == 0 || (order == 1 && (tile == TILE_16x8 || tile == TILE_32x8));
}

int fused_extra_planes(int tile) { return split_tile(tile) ? 5 : 4; }

int64_t fused_num_blocks(const Consts &c, int tile, int zchunk)
{
    int bx, by;
    tile_dims(tile, &bx, &by);
    return (int64_t)((c.nx + bx - 1) / bx) * ((c.ny + by - 1) / by) * ((c.nz + zchunk - 1) / zchunk);
}

hipError_t launch_fused_stage(const Consts &c, const StageArgs &s, ns_precision prec,
                              int tile, hipStream_t st)
{
    if (split_tile(tile)) return launch_split_stage(c, s, prec, tile, st);
    if (prec == NS_FP64)
        return launch_tile<double, double, double>(tile, c, s, st);
    // FP32 storage: stage 1 reads the double state, stage 3 writes it.
    if (s.mode == 1) return launch_tile<double, float, float>(tile, c, s, st);
    if (s.mode == 2) return launch_tile<float, float, float>(tile, c, s, st);
    return launch_tile<float, double, float>(tile, c, s, st);
}

}  // namespace ns
