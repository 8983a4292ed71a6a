// ns_split.hip -- the fused on-the-fly stage kernel with the work of each
// grid point split between two groups of waves.
//
// Same algorithm class and arithmetic as the one-thread-per-column kernel of
// ns_fused.hip (minimal storage: every derivative of the governing-equations
// section evaluated on the fly from an LDS-staged (x, y) tile marching along
// z, the low-storage RK3 update of the generic-algorithm figure in the same
// pass), but a block holds two threads per column of its tile:
//  * group M (threads [0, NT)) loads and stages each plane into LDS and
//    evaluates the three momentum equations;
//  * group E (threads [NT, 2 NT)) evaluates the mass and energy equations
//    and the viscous vector V_i = lap u_i + (1/3) d_i div u, which the
//    momentum equations need too.  E hands V to M through a small LDS buffer: in the
//    step of plane zp it writes the in-plane part of V at plane zp and the
//    z part at plane zp - 2, and M reads both one step later, after the
//    plane barrier.  So M finishes plane zp - 3 in that step, one plane
//    behind E.
// Each group keeps only its own equations' z-ring state, about half of the
// one-thread kernel's ring registers, so a block of 2 NT threads fits where
// NT threads of the one-thread kernel did not leave room for a second wave
// per SIMD, and the two groups' instruction streams hide each other's LDS
// and memory latency.
//
// The z-derivative handling (constant-coefficient fluxes scattered into a
// five-deep ring of pending residuals, point-value-weighted terms gathered
// from a ring of primitives, mixed derivatives as z derivatives of in-plane
// ones), the FP32 deviation storage format and the diagnostics of the stage
// input follow the one-thread kernel.  The in-plane mixed derivatives
// d_x d_y u and d_x d_y v differ: group E applies the x-stencil across the
// lanes of a tile row to the y-derivatives the lanes already hold (DPP wave
// shifts), where the one-thread kernel reads 16 LDS taps.
#include <type_traits>

#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

namespace {

template <typename TIN, typename CT>
__device__ __forceinline__ CT sp_to_ct(TIN v, double ref)
{
    if constexpr (std::is_same<CT, double>::value)
        return v;
    else if constexpr (std::is_same<TIN, double>::value)
        return (float)(v - ref);
    else
        return v;
}

// Stage outputs and the accumulator are touched once per stage: streamed
// past L2 so they do not displace the input planes that neighbouring blocks
// read again as halo.
template <typename TOUT>
__device__ __forceinline__ void sp_store(void *q, int64_t i, double v, double ref)
{
    if constexpr (std::is_same<TOUT, double>::value)
        __builtin_nontemporal_store(v, (double *)q + i);
    else
        __builtin_nontemporal_store((float)(v - ref), (float *)q + i);
}

// 1/x: hardware estimate and Newton steps r <- r + r (1 - x r); two steps
// reach double rounding error, one single.  x (a density) is positive and
// normal.
__device__ __forceinline__ double sp_recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float sp_recip(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

template <int V>
using SIC = std::integral_constant<int, V>;

}  // namespace

// MODE: 0 = residual only (R to s.rout), 1..3 = RK stage.
// PAIR (even nx): group M loads the halo plane two
// x-neighbours per lane with one 2-wide load and stages them with one
// 2-wide LDS store per field; pairs start at even x, so with nx even they
// never straddle the periodic wrap.
//
// Work split.  Group M (loads, staging, momentum) finishes plane zp - 3 in
// the step of plane zp; group E (mass, energy, viscous vector) finishes
// plane zp - 2 and hands M the viscous vector through vbuf.  Every lane
// computes, whether or not its column lies inside the grid (its LDS cells
// hold wrapped, valid values); only global stores and diagnostics are
// masked.  (The range checks of the march stay scalar branches: without them
// a five-plane chunk becomes one basic block that the register allocator
// cannot fit in 256 VGPRs.)
template <int BX, int BY, typename TIN, typename TOUT, typename CT, int MODE, bool DIAG, bool PAIR>
__global__ void __launch_bounds__(2 * BX * BY)
split_stage_kernel(Consts c, StageArgs s)
{
    // Multiply-adds are fused only within one expression, never across
    // statements: the march's five phases are compiled separately, and
    // fusion across statements can differ between them, which would make a
    // point's rounding depend on where its plane falls in a z-chunk.
#pragma clang fp contract(on)
    static_assert(MODE != 1 || std::is_same<TIN, double>::value, "stage 1 reads the double state");
    static_assert(!DIAG || MODE == 1, "diagnostics of the step's input state are taken in stage 1");
    static_assert(BX % 2 == 0, "pairs need an even tile width");
    constexpr bool DEV = std::is_same<CT, float>::value;
    constexpr int HX = BX + 4, HY = BY + 4, HP = HX * HY, NT = BX * BY;
    static_assert(HP % 2 == 0, "pair cells start at even LDS offsets");
    constexpr int PW = PAIR ? 2 : 1;                        // points per load slot
    constexpr int NLOAD = (HP + PW * NT - 1) / (PW * NT);
    constexpr int NW = 2 * NT / 64;
    static_assert(NT % 64 == 0, "each group must be whole waves");
    enum { L_RHO, L_M0, L_M1, L_M2, L_E, L_U, L_V, L_W, L_P, L_T, NF };
    __shared__ __attribute__((aligned(16))) CT lds[2][NF][HP];
    // E -> M: (V_x, V_y, V_z) in-plane part at plane zp, z part at plane zp - 2
    __shared__ CT vbuf[2][6][NT];
    __shared__ double red[NW][kDiag];

    // The group is a property of the wave; reading it through a scalar
    // register makes the branch below a scalar branch, so each wave runs
    // exactly one group's march (and its barriers).
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const bool grp_e = wave >= NT / 64;
    const int pt = (int)threadIdx.x - (grp_e ? NT : 0);
    const int tx = pt % BX, ty = pt / BX;
    int tbx, tby, tbz;
    xcd_tile(&tbx, &tby, &tbz);
    const int x0 = tbx * BX, y0 = tby * BY;
    const int z0 = tbz * s.zchunk;
    const int z1 = min(z0 + s.zchunk, c.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = (gx < c.nx) && (gy < c.ny);
    const int own = (ty + 2) * HX + tx + 2;
    const int64_t N = c.N;
    const int64_t col = active ? (int64_t)gy * c.nx + gx : 0;

    const CT c1x = (CT)c.c1[0], c1y = (CT)c.c1[1], c1z = (CT)c.c1[2];
    const CT c2x = (CT)c.c2[0], c2y = (CT)c.c2[1], c2z = (CT)c.c2[2];
    const CT inv_re = (CT)c.inv_re, kappa = (CT)c.kappa;
    const CT gm1 = (CT)c.gm1, gM2 = (CT)c.gM2;
    const CT half = CT(0.5), third = CT(1) / CT(3), four3 = CT(4) / CT(3);
    const CT two3 = CT(2) / CT(3);
    const CT kz = kappa * c2z;

    // per-column diagnostic sums of stage 1 with diagnostics, added in
    // program order (deterministic): group M the three momenta, group E mass,
    // energy, kinetic energy and enstrophy
    double dr[4] = {0.0, 0.0, 0.0, 0.0};

    // The march covers planes z0-2 .. z1+2 (M finishes a plane three steps
    // after loading it), padded to a multiple of 5; padding planes are
    // loaded (wrapped, valid memory) but never output.
    const int L = z1 - z0 + 5;

#define LV(f, dy, dx) lds[b][f][own + (dy) * HX + (dx)]
#define DX1(f) d1u(LV(f, 0, -2), LV(f, 0, -1), LV(f, 0, 1), LV(f, 0, 2))
#define DY1(f) d1u(LV(f, -2, 0), LV(f, -1, 0), LV(f, 1, 0), LV(f, 2, 0))
#define DX1P(f, g)                                                       \
    d1u(LV(f, 0, -2) * LV(g, 0, -2), LV(f, 0, -1) * LV(g, 0, -1),        \
        LV(f, 0, 1) * LV(g, 0, 1), LV(f, 0, 2) * LV(g, 0, 2))
#define DY1P(f, g)                                                       \
    d1u(LV(f, -2, 0) * LV(g, -2, 0), LV(f, -1, 0) * LV(g, -1, 0),        \
        LV(f, 1, 0) * LV(g, 1, 0), LV(f, 2, 0) * LV(g, 2, 0))
#define HF(dy, dx, g) ((half * LV(L_E, dy, dx) + LV(L_P, dy, dx)) * LV(g, dy, dx))
#define DX1H() d1u(HF(0, -2, L_U), HF(0, -1, L_U), HF(0, 1, L_U), HF(0, 2, L_U))
#define DY1H() d1u(HF(-2, 0, L_V), HF(-1, 0, L_V), HF(1, 0, L_V), HF(2, 0, L_V))
#define DX2(f) d2u(LV(f, 0, -2), LV(f, 0, -1), LV(f, 0, 0), LV(f, 0, 1), LV(f, 0, 2))
#define DY2(f) d2u(LV(f, -2, 0), LV(f, -1, 0), LV(f, 0, 0), LV(f, 1, 0), LV(f, 2, 0))

    if (!grp_e) {
        // ------------------------------------------------------------ group M
        const TIN *qin = (const TIN *)s.qin;
        enum { Z_M0, Z_M1, Z_M2, Z_W, NZ };
        CT qz[5][NZ];      // ring: rho u, rho v, rho w, w of the own column
        CT ra[5][3];       // ring: pending momentum residuals
        CT rp[3];          // plane zp - 2 with its z terms, V still missing
        TIN pf[NLOAD][5][PW];  // plane zp + 1, staged in step zp
        TIN pg[NLOAD][5][PW];  // plane zp + 2, loaded in step zp
        double acc[3];
        double accn[3];                // accumulator of the next step's point, prefetched
#pragma unroll
        for (int f = 0; f < 3; ++f) acc[f] = accn[f] = 0.0;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
#pragma unroll
            for (int f = 0; f < NZ; ++f) qz[q][f] = CT(0);
#pragma unroll
            for (int f = 0; f < 3; ++f) ra[q][f] = CT(0);
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) rp[f] = CT(0);

        // Plane offsets and LDS cells of the points this thread loads;
        // lcell < 0 marks an unused slot.
        int loff[NLOAD], lcell[NLOAD];
#pragma unroll
        for (int r = 0; r < NLOAD; ++r) {
            int lx = 0, ly = 0;
            lcell[r] = -1;
            if constexpr (PAIR) {
                const int q = pt + r * NT;          // pair index
                if (q < HP / 2) {
                    lx = 2 * (q % (HX / 2));
                    ly = q / (HX / 2);
                    lcell[r] = ly * HX + lx;
                }
            } else {
                const int idx = pt + r * NT;
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
        auto load_plane = [&](int zp, TIN (&dst)[NLOAD][5][PW]) {
            int zw = zp % c.nz;
            if (zw < 0) zw += c.nz;
            const int64_t base = (int64_t)zw * c.nxy;
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
        auto stage_plane = [&](int b) {
#pragma unroll
            for (int r = 0; r < NLOAD; ++r) {
                if (lcell[r] < 0) continue;
                CT val[NF][PW];
#pragma unroll
                for (int j = 0; j < PW; ++j) {
                    const CT rho = sp_to_ct<TIN, CT>(pf[r][0][j], c.rho_ref);
                    const CT m0 = sp_to_ct<TIN, CT>(pf[r][1][j], 0.0);
                    const CT m1 = sp_to_ct<TIN, CT>(pf[r][2][j], 0.0);
                    const CT m2 = sp_to_ct<TIN, CT>(pf[r][3][j], 0.0);
                    const CT E = sp_to_ct<TIN, CT>(pf[r][4][j], c.rhoE_ref);
                    const CT rhof = DEV ? CT(1) + rho : rho;
                    const CT inv = sp_recip(rhof);
                    const CT u = m0 * inv, v = m1 * inv, w = m2 * inv;
                    const CT p = gm1 * (E - half * (m0 * u + m1 * v + m2 * w));
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
                        // one 2-wide store per field: consecutive lanes
                        // write consecutive 2-point cells.  Indexing the
                        // row as an array of pairs (idx is even, rows start
                        // 16-byte aligned) lets the compiler use one
                        // 16-byte LDS store instead of two 8-byte halves.
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

        auto step = [&](auto phc, int zp) {
            constexpr int PH = decltype(phc)::value;
            constexpr int SM2 = (PH + 3) % 5, SM1 = (PH + 4) % 5, S0 = PH;
            constexpr int SP1 = (PH + 1) % 5, SP2 = (PH + 2) % 5;
            constexpr int SM4 = (PH + 1) % 5, SM3 = (PH + 2) % 5;
            const int b = (zp - z0) & 1;
            const int zf = zp - 3;
            const bool do_fin = (zf >= z0 && zf < z1);
            const bool do_plane = (zp >= z0 && zp < z1);
            const bool do_vin = (zp - 1 >= z0 && zp - 1 < z1);
            const int64_t pidx = (int64_t)(do_fin ? zf : z0) * c.nxy + col;
            // Plane zp + 2 and the accumulator of the next step's point are
            // loaded now, before this step's stores: vector memory counters
            // retire loads and stores in issue order, so a load issued after
            // a store could only be waited for together with that store.
            // Issued this way, the waits of the next step (staging plane
            // zp + 2, finishing plane zf + 1) never include this step's
            // stores.  Idle lanes read a valid address they ignore.
            load_plane(zp + 2, pg);
            if constexpr (MODE >= 1) {
                // stages 2 and 3 read the accumulator, stage 1 the state
                const double *src = (MODE >= 2) ? s.acc_in : (const double *)s.qin;
                const int zn = zf + 1;
                const int64_t pn = (int64_t)((zn >= z0 && zn < z1) ? zn : z0) * c.nxy + col;
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    acc[f] = accn[f];
                    accn[f] = __builtin_nontemporal_load(src + (1 + f) * N + pn);
                }
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) ra[SP2][f] = CT(0);

            {
                const CT m0 = LV(L_M0, 0, 0), m1 = LV(L_M1, 0, 0), m2 = LV(L_M2, 0, 0);
                const CT u = LV(L_U, 0, 0), v = LV(L_V, 0, 0), w = LV(L_W, 0, 0);
                const CT p = LV(L_P, 0, 0);
                qz[S0][Z_M0] = m0;
                qz[S0][Z_M1] = m1;
                qz[S0][Z_M2] = m2;
                qz[S0][Z_W] = w;

                const CT g0 = -half * c1z * (m0 * w);            // -1/2 d(rho u w)/dz
                const CT g1 = -half * c1z * (m1 * w);            // -1/2 d(rho v w)/dz
                const CT g2 = -c1z * (half * (m2 * w) + p);      // -1/2 d(rho w w)/dz - dp/dz
                const CT g[3] = {g0, g1, g2};
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    ra[SM2][f] -= g[f];
                    ra[SM1][f] += CT(8) * g[f];
                    ra[SP1][f] -= CT(8) * g[f];
                    ra[SP2][f] += g[f];
                }

                if (do_plane) {
                    const CT uc = u * c1x, vc = v * c1y;
                    const CT a = c1x * DX1(L_U) + c1y * DY1(L_V);
                    ra[S0][0] -= half * (c1x * DX1P(L_M0, L_U) + c1y * DY1P(L_M0, L_V) + m0 * a
                                         + uc * DX1(L_M0) + vc * DY1(L_M0))
                                 + c1x * DX1(L_P);
                    ra[S0][1] -= half * (c1x * DX1P(L_M1, L_U) + c1y * DY1P(L_M1, L_V) + m1 * a
                                         + uc * DX1(L_M1) + vc * DY1(L_M1))
                                 + c1y * DY1(L_P);
                    ra[S0][2] -= half * (c1x * DX1P(L_M2, L_U) + c1y * DY1P(L_M2, L_V) + m2 * a
                                         + uc * DX1(L_M2) + vc * DY1(L_M2));
                }
                // in-plane viscous part of plane zp - 1 (from E's last step)
                if (do_vin) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) ra[SM1][k] += inv_re * vbuf[b ^ 1][k][pt];
                }
            }

            // stage plane zp + 1 into the other LDS buffer (last read in the
            // previous step, before its barrier)
            stage_plane(b ^ 1);

            // finish plane zp - 3: z viscous part from E, RK update, output
            if (do_fin) {
                double Rd[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) Rd[k] = (double)(rp[k] + inv_re * vbuf[b ^ 1][3 + k][pt]);
                if (active) {
                    if constexpr (MODE == 0) {
#pragma unroll
                        for (int f = 0; f < 3; ++f) s.rout[(1 + f) * N + pidx] = Rd[f];
                    } else {
                        if constexpr (DIAG) {
#pragma unroll
                            for (int f = 0; f < 3; ++f) dr[f] += acc[f];
                        }
#pragma unroll
                        for (int f = 0; f < 3; ++f) {
                            sp_store<TOUT>(s.qout, (1 + f) * N + pidx, acc[f] + s.a_dt * Rd[f], 0.0);
                            if constexpr (MODE < 3)
                                __builtin_nontemporal_store(acc[f] + s.b_dt * Rd[f], s.acc_out + (1 + f) * N + pidx);
                        }
                    }
                }
            }

            // gathered z terms of plane zp - 2 (finished in the next step)
            {
#define DZ1(f) d1u(qz[SM4][f], qz[SM3][f], qz[SM1][f], qz[S0][f])
                const CT wc = qz[SM2][Z_W] * c1z;
                const CT Gzz = c1z * DZ1(Z_W);
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    rp[k] = ra[SM2][k] - half * (qz[SM2][Z_M0 + k] * Gzz + wc * DZ1(Z_M0 + k));
#undef DZ1
            }
#pragma unroll
            for (int r = 0; r < NLOAD; ++r)
#pragma unroll
                for (int f = 0; f < 5; ++f)
#pragma unroll
                    for (int j = 0; j < PW; ++j) pf[r][f][j] = pg[r][f][j];
            lds_barrier();
        };

        // prologue: plane z0 - 2 into LDS buffer 0
        load_plane(z0 - 2, pf);
        stage_plane(0);
        load_plane(z0 - 1, pf);
        lds_barrier();
        auto chunk = [&](int it) {
            const int zp = z0 - 2 + it;
            step(SIC<0>{}, zp);
            step(SIC<1>{}, zp + 1);
            step(SIC<2>{}, zp + 2);
            step(SIC<3>{}, zp + 3);
            step(SIC<4>{}, zp + 4);
        };
        for (int it = 0; it < L; it += 5) chunk(it);
    } else {
        // ------------------------------------------------------------ group E
        enum { Z_E, Z_U, Z_V, Z_W, Z_RHO, NZ };
        constexpr int R_EN = 0, R_MASS = 1;
        constexpr int NR = 2;
        CT qz[5][NZ];               // ring: rho E, u, v, w, rho of the own column
        CT qa[5], qb[5], qc[5];     // ring: D_x u + D_y v, D_x w, D_y w
        CT ra[5][NR];               // ring: pending energy and mass residuals
        double acc0 = 0.0, acc4 = 0.0;
        double accn0 = 0.0, accn4 = 0.0;    // next step's, prefetched
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            qa[q] = qb[q] = qc[q] = CT(0);
#pragma unroll
            for (int f = 0; f < NZ; ++f) qz[q][f] = CT(0);
#pragma unroll
            for (int f = 0; f < NR; ++f) ra[q][f] = CT(0);
        }

        auto step = [&](auto phc, int zp) {
            constexpr int PH = decltype(phc)::value;
            constexpr int SM2 = (PH + 3) % 5, SM1 = (PH + 4) % 5, S0 = PH;
            constexpr int SP1 = (PH + 1) % 5, SP2 = (PH + 2) % 5;
            constexpr int SM4 = (PH + 1) % 5, SM3 = (PH + 2) % 5;
            const int b = (zp - z0) & 1;
            const int zf = zp - 2;
            const bool do_fin = (zf >= z0 && zf < z1);
            const bool do_plane = (zp >= z0 && zp < z1);
            const int64_t pidx = (int64_t)(do_fin ? zf : z0) * c.nxy + col;
            if constexpr (MODE >= 1) {
                // one step ahead, as in group M
                const double *src = (MODE >= 2) ? s.acc_in : (const double *)s.qin;
                const int zn = zf + 1;
                const int64_t pn = (int64_t)((zn >= z0 && zn < z1) ? zn : z0) * c.nxy + col;
                acc0 = accn0;
                acc4 = accn4;
                accn0 = __builtin_nontemporal_load(src + pn);
                accn4 = __builtin_nontemporal_load(src + 4 * N + pn);
            }
#pragma unroll
            for (int f = 0; f < NR; ++f) ra[SP2][f] = CT(0);

            {
                const CT E = LV(L_E, 0, 0), rho = LV(L_RHO, 0, 0);
                const CT u = LV(L_U, 0, 0), v = LV(L_V, 0, 0), w = LV(L_W, 0, 0);
                const CT p = LV(L_P, 0, 0), T = LV(L_T, 0, 0), m2 = LV(L_M2, 0, 0);
                const CT dyu = DY1(L_U), dyv = DY1(L_V);
                const CT Gxx = c1x * DX1(L_U), Gxy = c1y * dyu;
                const CT Gyx = c1x * DX1(L_V), Gyy = c1y * dyv;
                const CT Gzx = c1x * DX1(L_W), Gzy = c1y * DY1(L_W);
                const CT a = Gxx + Gyy;
                qz[S0][Z_E] = E;
                qz[S0][Z_U] = u;
                qz[S0][Z_V] = v;
                qz[S0][Z_W] = w;
                qz[S0][Z_RHO] = rho;
                qa[S0] = a;
                qb[S0] = Gzx;
                qc[S0] = Gzy;

                const CT g4 = -c1z * ((half * E + p) * w);   // -1/2 d(rhoE w)/dz - d(p w)/dz
                const CT gT = kz * T;                        // kappa d2T/dz2
                const CT g0 = -half * c1z * m2;              // -1/2 d(rho w)/dz
                ra[SM2][R_EN] -= g4;
                ra[SM1][R_EN] += CT(8) * g4;
                ra[SP1][R_EN] -= CT(8) * g4;
                ra[SP2][R_EN] += g4;
                ra[SM2][R_EN] -= gT;
                ra[SM1][R_EN] += CT(16) * gT;
                ra[S0][R_EN] -= CT(30) * gT;
                ra[SP1][R_EN] += CT(16) * gT;
                ra[SP2][R_EN] -= gT;
                ra[SM2][R_MASS] -= g0;
                ra[SM1][R_MASS] += CT(8) * g0;
                ra[SP1][R_MASS] -= CT(8) * g0;
                ra[SP2][R_MASS] += g0;

                if (do_plane) {
                    const CT uc = u * c1x, vc = v * c1y;
                    // mixed derivatives d_x d_y v and d_x d_y u: the x-stencil
                    // applied across the row's lanes to the y-derivatives
                    // they already hold; a row's two end lanes on each side
                    // take the y-derivative at their halo column (x - 2 at
                    // the start of the row, x + 2 at its end).  The other
                    // lanes read their own column, which keeps the wave's
                    // addresses on distinct LDS banks.
                    const int hx = (tx < 2) ? -2 : (tx >= BX - 2 ? 2 : 0);
#define LVH(f, dy) lds[b][f][own + (dy) * HX + hx]
                    const CT hu = d1u(LVH(L_U, -2), LVH(L_U, -1), LVH(L_U, 1), LVH(L_U, 2));
                    const CT hv = d1u(LVH(L_V, -2), LVH(L_V, -1), LVH(L_V, 1), LVH(L_V, 2));
#undef LVH
                    const CT dxdyv = d1u_x_lanes<BX>(dyv, hv, tx);
                    const CT dxdyu = d1u_x_lanes<BX>(dyu, hu, tx);
                    // d_j tau_ij = lap u_i + (1/3) d_i div u, in-plane parts
                    const CT Vx = four3 * (c2x * DX2(L_U)) + c2y * DY2(L_U)
                                  + third * (c1x * c1y * dxdyv);
                    const CT Vy = c2x * DX2(L_V) + four3 * (c2y * DY2(L_V))
                                  + third * (c1x * c1y * dxdyu);
                    const CT Vz = c2x * DX2(L_W) + c2y * DY2(L_W);
                    vbuf[b][0][pt] = Vx;
                    vbuf[b][1][pt] = Vy;
                    vbuf[b][2][pt] = Vz;
                    // tau_ij du_i/dx_j restricted to terms without a z derivative
                    const CT phi = CT(2) * (Gxx * Gxx + Gyy * Gyy) + Gxy * Gxy + Gyx * Gyx
                                   + CT(2) * Gxy * Gyx + Gzx * Gzx + Gzy * Gzy;
                    const CT rhof = DEV ? CT(1) + rho : rho;
                    if constexpr (DEV) {
                        ra[S0][R_MASS] -= half * (c1x * DX1(L_M0) + c1y * DY1(L_M1) + rhof * a
                                                  + uc * DX1(L_RHO) + vc * DY1(L_RHO));
                    } else {
                        // rho u and rho v at the taps, from the rho and
                        // velocity taps this group reads anyway (equal to
                        // the staged momenta up to rounding)
                        ra[S0][R_MASS] -= half * (c1x * DX1P(L_RHO, L_U) + c1y * DY1P(L_RHO, L_V)
                                                  + rhof * a + uc * DX1(L_RHO) + vc * DY1(L_RHO));
                    }
                    if constexpr (DIAG) {
                        // the kinetic energy and the omega_z part of the
                        // enstrophy are complete in the plane; the vorticity
                        // components with z derivatives are added when the
                        // point is finished
                        const double oz = (double)(Gyx - Gxy);
                        const double rd = (double)rhof;
                        if (active) {
                            dr[2] += 0.5 * rd * ((double)u * (double)u + (double)v * (double)v
                                                + (double)w * (double)w);
                            dr[3] += 0.5 * rd * oz * oz;
                        }
                    }
                    ra[S0][R_EN] += -(c1x * DX1H() + c1y * DY1H())
                                    - half * (E * a + uc * DX1(L_E) + vc * DY1(L_E))
                                    + inv_re * (u * Vx + v * Vy + w * Vz + phi)
                                    + kappa * (c2x * DX2(L_T) + c2y * DY2(L_T));
                }
            }

            // finish plane zf = zp - 2: gathered z terms, RK update, output
            if (do_fin) {
#define DZ1(f) d1u(qz[SM4][f], qz[SM3][f], qz[SM1][f], qz[S0][f])
#define DZ2(f) d2u(qz[SM4][f], qz[SM3][f], qz[SM2][f], qz[SM1][f], qz[S0][f])
                const CT E = qz[SM2][Z_E], rho = qz[SM2][Z_RHO];
                const CT u = qz[SM2][Z_U], v = qz[SM2][Z_V], w = qz[SM2][Z_W];
                const CT rhof = DEV ? CT(1) + rho : rho;
                const CT a = qa[SM2], bb = qb[SM2], cc = qc[SM2];
                const CT wc = w * c1z;
                const CT Gxz = c1z * DZ1(Z_U), Gyz = c1z * DZ1(Z_V), Gzz = c1z * DZ1(Z_W);
                const CT Da = c1z * d1u(qa[SM4], qa[SM3], qa[SM1], qa[S0]);
                const CT Db = c1z * d1u(qb[SM4], qb[SM3], qb[SM1], qb[S0]);
                const CT Dc = c1z * d1u(qc[SM4], qc[SM3], qc[SM1], qc[S0]);
                const CT Vx = c2z * DZ2(Z_U) + third * Db;
                const CT Vy = c2z * DZ2(Z_V) + third * Dc;
                const CT Vz = four3 * (c2z * DZ2(Z_W)) + third * Da;
                vbuf[b][3][pt] = Vx;
                vbuf[b][4][pt] = Vy;
                vbuf[b][5][pt] = Vz;
                const CT div = a + Gzz;
                const CT phi = Gxz * Gxz + Gyz * Gyz + CT(2) * Gzz * Gzz
                               + CT(2) * (Gxz * bb + Gyz * cc) - two3 * div * div;
                const CT R4 = ra[SM2][R_EN] - half * (E * Gzz + wc * DZ1(Z_E))
                              + inv_re * (u * Vx + v * Vy + w * Vz + phi);
                const CT R0 = ra[SM2][R_MASS] - half * (rhof * Gzz + wc * DZ1(Z_RHO));
                double Rd4 = (double)R4;
                if constexpr (DEV) Rd4 -= c.H_ref * ((double)a + (double)Gzz);
                const double Rd0 = (double)R0;
                if (active) {
                    if constexpr (MODE == 0) {
                        s.rout[pidx] = Rd0;
                        s.rout[4 * N + pidx] = Rd4;
                    } else {
                        if constexpr (DIAG) {
                            const CT ox = cc - Gyz, oy = Gxz - bb;
                            dr[0] += acc0;
                            dr[1] += acc4;
                            dr[3] += 0.5 * (double)rhof * ((double)ox * (double)ox + (double)oy * (double)oy);
                        }
                        sp_store<TOUT>(s.qout, pidx, acc0 + s.a_dt * Rd0, c.rho_ref);
                        sp_store<TOUT>(s.qout, 4 * N + pidx, acc4 + s.a_dt * Rd4, c.rhoE_ref);
                        if constexpr (MODE < 3) {
                            __builtin_nontemporal_store(acc0 + s.b_dt * Rd0, s.acc_out + pidx);
                            __builtin_nontemporal_store(acc4 + s.b_dt * Rd4, s.acc_out + 4 * N + pidx);
                        }
                    }
                }
#undef DZ1
#undef DZ2
            }
            lds_barrier();
        };

        // prologue: matches group M's barrier
        lds_barrier();
        auto chunk = [&](int it) {
            const int zp = z0 - 2 + it;
            step(SIC<0>{}, zp);
            step(SIC<1>{}, zp + 1);
            step(SIC<2>{}, zp + 2);
            step(SIC<3>{}, zp + 3);
            step(SIC<4>{}, zp + 4);
        };
        for (int it = 0; it < L; it += 5) chunk(it);
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

    if constexpr (DIAG) {
        // block reduction of the diagnostic partial sums, fixed order: each
        // thread takes the column sums of its own group's slots (the other
        // group's slots count zero for it), then waves, then the block
        const int tid = threadIdx.x;
        __syncthreads();
        double dsum[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (grp_e) {
            dsum[0] = dr[0];
            dsum[4] = dr[1];
            dsum[5] = dr[2];
            dsum[6] = dr[3];
        } else {
            dsum[1] = dr[0];
            dsum[2] = dr[1];
            dsum[3] = dr[2];
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            double vsum = dsum[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) vsum += __shfl_xor(vsum, off, 64);
            dsum[k] = vsum;
        }
        if ((tid & 63) == 0) {
#pragma unroll
            for (int k = 0; k < 7; ++k) red[tid >> 6][k] = dsum[k];
        }
        __syncthreads();
        if (tid == 0) {
            const int64_t blin = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            for (int k = 0; k < 7; ++k) {
                double t = 0.0;
                for (int wv = 0; wv < NW; ++wv) t += red[wv][k];
                s.diag_partial[blin * kDiag + k] = t;
            }
            s.diag_partial[blin * kDiag + 7] = 0.0;
        }
    }
}

namespace {

template <int BX, int BY, typename TIN, typename TOUT, typename CT, int MODE, bool DIAG, bool PAIR>
void launch_one(const Consts &c, const StageArgs &s, hipStream_t st)
{
    dim3 block(2 * BX * BY, 1, 1);
    dim3 grid((c.nx + BX - 1) / BX, (c.ny + BY - 1) / BY, (c.nz + s.zchunk - 1) / s.zchunk);
    hipLaunchKernelGGL((split_stage_kernel<BX, BY, TIN, TOUT, CT, MODE, DIAG, PAIR>), grid, block, 0, st,
                       c, s);
}

// The halo plane is loaded in x-neighbour pairs when nx is even.
template <int BX, int BY, typename TIN, typename TOUT, typename CT, int MODE>
hipError_t launch_mode(const Consts &c, const StageArgs &s, hipStream_t st)
{
    const bool pair = c.nx % 2 == 0;
    if constexpr (MODE == 1) {
        if (s.diag_partial != nullptr) {
            if (pair) launch_one<BX, BY, TIN, TOUT, CT, 1, true, true>(c, s, st);
            else launch_one<BX, BY, TIN, TOUT, CT, 1, true, false>(c, s, st);
            return hipGetLastError();
        }
    }
    if (pair)
        launch_one<BX, BY, TIN, TOUT, CT, MODE, false, true>(c, s, st);
    else
        launch_one<BX, BY, TIN, TOUT, CT, MODE, false, false>(c, s, st);
    return hipGetLastError();
}

template <typename TIN, typename TOUT, typename CT, int MODE>
hipError_t launch_sp_tile(int tile, const Consts &c, const StageArgs &s, hipStream_t st)
{
    switch (tile) {
    case TILE_16x8_2G: return launch_mode<16, 8, TIN, TOUT, CT, MODE>(c, s, st);
    case TILE_32x8_2G: return launch_mode<32, 8, TIN, TOUT, CT, MODE>(c, s, st);
    case TILE_16x4_2G: return launch_mode<16, 4, TIN, TOUT, CT, MODE>(c, s, st);
    default: return hipErrorInvalidValue;
    }
}

template <int BX, int BY, typename T>
int resident_sp()
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(&split_stage_kernel<BX, BY, T, T, T, 2, false, true>),
            2 * BX * BY, 0) != hipSuccess)
        return 0;
    return cus * (per > 0 ? per : 1);
}

}  // namespace

bool split_tile(int tile) { return tile == TILE_16x8_2G || tile == TILE_32x8_2G || tile == TILE_16x4_2G; }

int split_resident_blocks(ns_precision prec, int tile)
{
    const bool d = prec == NS_FP64;
    switch (tile) {
    case TILE_16x8_2G: return d ? resident_sp<16, 8, double>() : resident_sp<16, 8, float>();
    case TILE_32x8_2G: return d ? resident_sp<32, 8, double>() : resident_sp<32, 8, float>();
    case TILE_16x4_2G: return d ? resident_sp<16, 4, double>() : resident_sp<16, 4, float>();
    default: return 0;
    }
}

hipError_t launch_split_stage(const Consts &c, const StageArgs &s, ns_precision prec, int tile,
                              hipStream_t st)
{
    if (prec == NS_FP64) {
        switch (s.mode) {
        case 0: return launch_sp_tile<double, double, double, 0>(tile, c, s, st);
        case 1: return launch_sp_tile<double, double, double, 1>(tile, c, s, st);
        case 2: return launch_sp_tile<double, double, double, 2>(tile, c, s, st);
        case 3: return launch_sp_tile<double, double, double, 3>(tile, c, s, st);
        default: return hipErrorInvalidValue;
        }
    }
    // FP32 storage: stage 1 reads the double state, stage 3 writes it.
    switch (s.mode) {
    case 1: return launch_sp_tile<double, float, float, 1>(tile, c, s, st);
    case 2: return launch_sp_tile<float, float, float, 2>(tile, c, s, st);
    case 3: return launch_sp_tile<float, double, float, 3>(tile, c, s, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ns
