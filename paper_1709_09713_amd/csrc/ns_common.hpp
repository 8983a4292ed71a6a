// ns_common.hpp -- shared device-side definitions of the HIP library.
//
// Grid constants are folded on the host once per call (the paper evaluates
// rationals and inverses of constants up front so that the loops contain no
// divisions: end of the algorithms section).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ns_tgv.h"

namespace ns {

// Conserved-variable slots in a state, field-major.
enum { F_RHO = 0, F_M0 = 1, F_M1 = 2, F_M2 = 3, F_E = 4 };

// Number of doubles in one diagnostics record / per-block partial.
constexpr int kDiag = 8;

struct Consts {
    int nx, ny, nz;
    int nxy;
    int64_t N;          // points per field
    double c1[3];       // 1 / (12 h_d): scale of the unscaled first-derivative stencil
    double c2[3];       // 1 / (12 h_d^2): scale of the unscaled second-derivative stencil
    double gm1;         // gamma - 1
    double gM2;         // gamma M^2
    double inv_re;      // 1 / Re (0 when inviscid)
    double kappa;       // 1 / ((gamma - 1) M^2 Pr Re)
    // Uniform reference state used by the FP32 storage format:
    // rho_ref = 1, p_ref = 1/(gamma M^2), rhoE_ref = p_ref/(gamma - 1).
    double rho_ref, p_ref, rhoE_ref, H_ref;   // H_ref = rhoE_ref + p_ref
    double vol;         // hx hy hz
    double inv_npts;    // 1 / N
};

Consts make_consts(const ns_params *p);

// Two-register low-storage RK3 (generic-algorithm figure): per stage k,
// Q = Q_acc + a_k dt R and Q_acc += b_k dt R; a = (2/3, 5/12, 3/5),
// b = (1/4, 3/20, 3/5).
__host__ __device__ constexpr double rk_a(int k)
{
    return k == 0 ? 2.0 / 3.0 : (k == 1 ? 5.0 / 12.0 : 3.0 / 5.0);
}
__host__ __device__ constexpr double rk_b(int k)
{
    return k == 0 ? 1.0 / 4.0 : (k == 1 ? 3.0 / 20.0 : 3.0 / 5.0);
}

__host__ __device__ inline int wrap1(int i, int n)
{
    // single wrap: valid for -n <= i < 2n
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Unscaled fourth-order first-derivative stencil (equation fd, times 12h):
//   (f[-2] - f[+2]) + 8 (f[+1] - f[-1]).
template <typename T>
__device__ __forceinline__ T d1u(T fm2, T fm1, T fp1, T fp2)
{
    return (fm2 - fp2) + T(8) * (fp1 - fm1);
}

// Unscaled fourth-order second-derivative stencil (equation sd, times 12h^2):
//   16 (f[-1] + f[+1]) - (f[-2] + f[+2]) - 30 f[0].
template <typename T>
__device__ __forceinline__ T d2u(T fm2, T fm1, T f0, T fp1, T fp2)
{
    return T(16) * (fm1 + fp1) - (fm2 + fp2) - T(30) * f0;
}

// Cross-lane moves of a per-lane value by one lane within the 64-wide wave
// (DPP wave shifts): lane_prev gives lane i the value of lane i - 1,
// lane_next that of lane i + 1.  A lane with no source lane (lane 0, resp.
// lane 63) gets 0.  Every lane of the wave must be active.  Doubles move as
// two 32-bit halves; the bits are copied exactly.
__device__ __forceinline__ int dpp_wave_shr1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_wave_shl1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(dpp_wave_shr1(__float_as_int(v))); }
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(dpp_wave_shl1(__float_as_int(v))); }
__device__ __forceinline__ double lane_prev(double v)
{
    return __hiloint2double(dpp_wave_shr1(__double2hiint(v)), dpp_wave_shr1(__double2loint(v)));
}
__device__ __forceinline__ double lane_next(double v)
{
    return __hiloint2double(dpp_wave_shl1(__double2hiint(v)), dpp_wave_shl1(__double2loint(v)));
}

// x-derivative (unscaled eq. fd) of a per-column value y that every lane of
// a tile row holds, for tile rows of BX lanes laid out along the wave (BX
// divides 64).  The four x-neighbours come from neighbouring lanes; the two
// lanes at each end of a row take the values they lack from h, which the
// first two lanes of a row (tx 0, 1) hold for column x - 2 and the last two
// (tx BX-2, BX-1) for column x + 2.  The other lanes' h is not used.
template <int BX, typename T>
__device__ __forceinline__ T d1u_x_lanes(T y, T h, int tx)
{
    static_assert(BX >= 4 && 64 % BX == 0, "tile rows must tile the wave, two lanes per end");
    const T p1 = lane_prev(y), p2 = lane_prev(p1);
    const T n1 = lane_next(y), n2 = lane_next(n1);
    const T hn = lane_next(h), hp = lane_prev(h);
    const T ym2 = tx >= 2 ? p2 : h;             // x - 2
    const T ym1 = tx >= 1 ? p1 : hn;            // x - 1 (row start: lane 1's x - 2)
    const T yp1 = tx <= BX - 2 ? n1 : hp;       // x + 1 (row end: lane BX-2's x + 2)
    const T yp2 = tx <= BX - 3 ? n2 : h;        // x + 2
    return d1u(ym2, ym1, yp1, yp2);
}

// XCD-aware tile order.  The dispatcher hands workgroups to the 8 XCDs
// round-robin by linear workgroup id, and each XCD has its own L2.  Remap so
// that XCD k processes the k-th contiguous run of tiles (x fastest, then y,
// then z): tiles that share halo rows and columns then run at the same time
// on the same L2.  Bijective for any grid size.
constexpr int kNumXcd = 8;

__device__ __forceinline__ void xcd_tile(int *bx, int *by, int *bz)
{
    const int gx = gridDim.x, gy = gridDim.y;
    const int total = gx * gy * gridDim.z;
    const int L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int k = L % kNumXcd, slot = L / kNumXcd;
    const int q = total / kNumXcd, r = total % kNumXcd;
    const int T = k * q + min(k, r) + slot;
    *bx = T % gx;
    *by = (T / gx) % gy;
    *bz = T / (gx * gy);
}

// Workgroup barrier that orders LDS only.  __syncthreads() is a release /
// acquire fence over all address spaces, which makes every wave wait for its
// outstanding global stores before the barrier; the stencil kernels only
// need their LDS writes to be visible to the other waves of the block.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace ns

#define NS_HIP_OK(expr)                                       \
    do {                                                      \
        if ((expr) != hipSuccess) return NS_ERR_DEVICE;       \
    } while (0)
