// ns_api.hip -- the C ABI (include/ns_tgv.h): argument validation,
// workspace layout and the per-step launch sequence of the three algorithm
// classes.  Every call validates first and enqueues nothing on failure.
#include <cmath>
#include <cstring>

#include "ns_common.hpp"
#include "ns_kernels.hpp"

namespace ns {

Consts make_consts(const ns_params *p)
{
    Consts c;
    c.nx = p->n[0];
    c.ny = p->n[1];
    c.nz = p->n[2];
    c.nxy = c.nx * c.ny;
    c.N = (int64_t)c.nxy * c.nz;
    double h[3];
    for (int d = 0; d < 3; ++d) {
        h[d] = p->length[d] / p->n[d];
        c.c1[d] = 1.0 / (12.0 * h[d]);
        c.c2[d] = 1.0 / (12.0 * h[d] * h[d]);
    }
    c.gm1 = p->gamma - 1.0;
    c.gM2 = p->gamma * p->mach * p->mach;
    c.inv_re = 1.0 / p->reynolds;   // 0 for +INFINITY
    c.kappa = 1.0 / (c.gm1 * p->mach * p->mach * p->prandtl * p->reynolds);
    c.rho_ref = 1.0;
    c.p_ref = 1.0 / c.gM2;
    c.rhoE_ref = c.p_ref / c.gm1;
    c.H_ref = c.rhoE_ref + c.p_ref;
    c.vol = h[0] * h[1] * h[2];
    c.inv_npts = 1.0 / (double)c.N;
    return c;
}


constexpr int kMinZChunk = 1;
// Launch settings of ns_set_fused_config / ns_set_fused_order: one copy per
// calling thread, so threads that drive solves of different shapes do not
// see each other's settings.
static thread_local int g_tile = -1;
static thread_local int g_zchunk = 0;
static thread_local int g_order = 0;

// Default z-chunk: a block marches zchunk + 4 planes (+ 5 for the
// two-group tiles; padded to the unroll of 5), and the grid runs in ceil(blocks / resident) rounds of resident
// blocks, so the time of a stage goes as rounds x padded planes.  Pick the
// number of chunks along z that minimises it (fewest blocks on a tie).
// resident = blocks the device holds at once (512 on MI355X for the default
// tiles); when it cannot be queried, 512 is assumed.
static int default_zchunk(const Consts &c, ns_precision prec, int tile)
{
    int bx, by;
    tile_dims(tile, &bx, &by);
    const int64_t nxy = (int64_t)((c.nx + bx - 1) / bx) * ((c.ny + by - 1) / by);
    int64_t resident = fused_resident_blocks(prec, tile);
    if (resident <= 0) resident = 512;
    int best_z = c.nz;
    int64_t best_cost = -1;
    for (int k = 1; k <= c.nz / kMinZChunk; ++k) {
        const int z = (c.nz + k - 1) / k;
        const int chunks = (c.nz + z - 1) / z;
        if (chunks != k) continue;   // the same z as a smaller k
        const int64_t rounds = (chunks * nxy + resident - 1) / resident;
        const int64_t planes = ((z + fused_extra_planes(tile) + 4) / 5) * 5;
        const int64_t cost = rounds * planes;
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best_z = z;
        }
    }
    return best_z;
}

// Launch shape: an explicit tile (>= 0) / zchunk (> 0) wins, else the
// calling thread's setting of ns_set_fused_config, else the default.
static void choose_config(const Consts &c, ns_precision prec, int tile_in, int zchunk_in, int *tile,
                          int *zchunk)
{
    int t = tile_in >= 0 ? tile_in : g_tile;
    int z = tile_in >= 0 ? zchunk_in : g_zchunk;
    if (zchunk_in > 0) z = zchunk_in;
    // defaults measured on MI355X: FP64 runs fastest with the two-group
    // 32x8 kernel on cubes from 128^3 to 512^3 (384^3: within 1% of the
    // one-thread 16x8 kernel), FP32 storage with the one-thread 32x8 kernel
    if (t < 0 || t >= TILE_COUNT) t = (prec == NS_FP64) ? TILE_32x8_2G : TILE_32x8;
    if (z <= 0) z = default_zchunk(c, prec, t);
    if (z < kMinZChunk) z = kMinZChunk;
    if (z > c.nz) z = c.nz;
    *tile = t;
    *zchunk = z;
}

static void choose_config(const Consts &c, ns_precision prec, int *tile, int *zchunk)
{
    choose_config(c, prec, -1, 0, tile, zchunk);
}

static int64_t max_partial_blocks(const Consts &c)
{
    int64_t m = diag_num_blocks(c);
    for (int t = 0; t < TILE_COUNT; ++t) {
        const int64_t b = fused_num_blocks(c, t, kMinZChunk);
        if (b > m) m = b;
    }
    return m;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t partial, rec, acc, b1, b2, R, stored, G, total;
};

// Scratch layout.  The diagnostic partials and one ns_diag record come
// first, so every workspace size returned by ns_workspace_bytes also serves
// diagnostics().
static Layout layout(const Consts &c, ns_algo algo, ns_precision prec)
{
    Layout L;
    size_t off = 0;
    const size_t n5 = 5 * (size_t)c.N;
    L.partial = off;
    off = align256(off + (size_t)max_partial_blocks(c) * kDiag * sizeof(double));
    L.rec = off;
    off = align256(off + sizeof(ns_diag));
    const size_t stage_elt = (prec == NS_FP64) ? sizeof(double) : sizeof(float);
    L.acc = off;
    off = align256(off + n5 * sizeof(double));
    L.b1 = off;
    off = align256(off + n5 * stage_elt);
    L.b2 = off;
    off = align256(off + n5 * stage_elt);
    L.R = L.stored = L.G = 0;
    if (algo == NS_ALGO_SOME) {
        L.G = off;
        off = align256(off + rs_workspace_doubles(c) * sizeof(double));
    }
    if (algo == NS_ALGO_STORED) {
        L.R = off;
        off = align256(off + n5 * sizeof(double));
        L.stored = off;
        off = align256(off + stored_workspace_doubles(c) * sizeof(double));
    }
    L.total = off;
    return L;
}

static size_t diag_bytes(const Consts &c)
{
    return align256((size_t)max_partial_blocks(c) * kDiag * sizeof(double)) + align256(sizeof(ns_diag));
}

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

static ns_status check_params(const ns_params *p)
{
    if (!p) return NS_ERR_ARG;
    int64_t n = 1;
    for (int d = 0; d < 3; ++d) {
        if (p->n[d] < 5 || p->n[d] > 2048) return NS_ERR_SHAPE;
        n *= p->n[d];
        if (!finite_pos(p->length[d])) return NS_ERR_ARG;
    }
    if (n >= ((int64_t)1 << 31)) return NS_ERR_SHAPE;
    if (!std::isfinite(p->gamma) || !(p->gamma > 1.0)) return NS_ERR_ARG;
    if (!finite_pos(p->prandtl) || !finite_pos(p->mach)) return NS_ERR_ARG;
    if (std::isnan(p->reynolds) || !(p->reynolds > 0.0)) return NS_ERR_ARG;
    return NS_OK;
}

ns_status validate_params(const ns_params *p) { return check_params(p); }

static bool valid_algo(int a) { return a == NS_ALGO_STORED || a == NS_ALGO_FUSED || a == NS_ALGO_SOME; }
static bool valid_prec(int q) { return q == NS_FP64 || q == NS_FP32_STORE; }

static ns_status check_work(const void *work, size_t have, size_t need)
{
    if (need > 0 && !work) return NS_ERR_ARG;
    if (have < need) return NS_ERR_WORKSPACE;
    if (((uintptr_t)work & 255) != 0) return NS_ERR_WORKSPACE;
    return NS_OK;
}

// State, Q and R arrays must be 16-byte aligned (the stage kernels load
// x-neighbour pairs of doubles with one 16-byte access); diagnostics
// records 8-byte aligned.
static bool aligned(const void *ptr, uintptr_t a) { return ((uintptr_t)ptr & (a - 1)) == 0; }

template <typename T>
static T *at(void *work, size_t off)
{
    return (T *)((char *)work + off);
}

ns_status make_fused_plan(const ns_params *p, ns_precision prec, int tile, int zchunk,
                          double *state, void *work, size_t work_bytes, FusedPlan *out)
{
    ns_status st = check_params(p);
    if (st != NS_OK) return st;
    if (!valid_prec(prec) || !state || !out || !aligned(state, 16)) return NS_ERR_ARG;
    if (tile < -1 || tile >= TILE_COUNT || zchunk < 0 || (zchunk > 0 && zchunk < kMinZChunk))
        return NS_ERR_ARG;
    const Consts c = make_consts(p);
    const Layout L = layout(c, NS_ALGO_FUSED, prec);
    st = check_work(work, work_bytes, L.total);
    if (st != NS_OK) return st;
    FusedPlan f;
    f.c = c;
    f.prec = prec;
    choose_config(c, prec, tile, zchunk, &f.tile, &f.zchunk);
    f.order = g_order;
    if (!fused_order_supported(f.tile, f.order)) return NS_ERR_UNSUPPORTED;
    f.nblk = fused_num_blocks(c, f.tile, f.zchunk);
    f.state = state;
    f.partial = at<double>(work, L.partial);
    f.acc = at<double>(work, L.acc);
    f.b1 = at<void>(work, L.b1);
    f.b2 = at<void>(work, L.b2);
    *out = f;
    return NS_OK;
}

// One RK3 step of the fused class: stage 1 Q^n -> b1 (next stage input)
// and the accumulator (plus the diagnostics partials of Q^n when diag_out
// is given, reduced into *diag_out right after), stage 2 b1 -> b2 with the
// accumulator in place, stage 3 b2 -> Q^{n+1} in the state buffer.
hipError_t enqueue_fused_step(const FusedPlan &f, double dt, ns_diag *diag_out, hipStream_t s)
{
    StageArgs a = {};
    a.zchunk = f.zchunk;
    a.order = f.order;
    a.qin = f.state;
    a.qout = f.b1;
    a.acc_out = f.acc;
    a.a_dt = rk_a(0) * dt;
    a.b_dt = rk_b(0) * dt;
    a.mode = 1;
    a.diag_partial = diag_out ? f.partial : nullptr;
    hipError_t e = launch_fused_stage(f.c, a, f.prec, f.tile, s);
    if (e != hipSuccess) return e;
    if (diag_out) {
        e = launch_diag_finalize(f.c, f.partial, f.nblk, diag_out, s);
        if (e != hipSuccess) return e;
    }
    a.qin = f.b1;
    a.acc_in = f.acc;
    a.acc_out = f.acc;
    a.qout = f.b2;
    a.a_dt = rk_a(1) * dt;
    a.b_dt = rk_b(1) * dt;
    a.mode = 2;
    a.diag_partial = nullptr;
    e = launch_fused_stage(f.c, a, f.prec, f.tile, s);
    if (e != hipSuccess) return e;
    a.qin = f.b2;
    a.acc_in = f.acc;
    a.acc_out = nullptr;
    a.qout = f.state;
    a.a_dt = rk_a(2) * dt;
    a.b_dt = 0.0;
    a.mode = 3;
    return launch_fused_stage(f.c, a, f.prec, f.tile, s);
}

}  // namespace ns

using namespace ns;

extern "C" {

const char *ns_status_string(ns_status s)
{
    switch (s) {
    case NS_OK: return "NS_OK";
    case NS_ERR_ARG: return "NS_ERR_ARG: invalid argument";
    case NS_ERR_SHAPE: return "NS_ERR_SHAPE: grid size out of range";
    case NS_ERR_WORKSPACE: return "NS_ERR_WORKSPACE: workspace too small or misaligned";
    case NS_ERR_DEVICE: return "NS_ERR_DEVICE: HIP error";
    case NS_ERR_NONFINITE: return "NS_ERR_NONFINITE: non-finite diagnostics";
    case NS_ERR_NOMEM: return "NS_ERR_NOMEM: device memory allocation failed";
    case NS_ERR_UNSUPPORTED: return "NS_ERR_UNSUPPORTED: combination not provided";
    }
    return "unknown ns_status";
}

size_t ns_state_bytes(const ns_params *p)
{
    if (check_params(p) != NS_OK) return 0;
    return 5 * (size_t)p->n[0] * p->n[1] * p->n[2] * sizeof(double);
}

size_t ns_workspace_bytes(const ns_params *p, ns_algo algo, ns_precision prec)
{
    if (check_params(p) != NS_OK || !valid_algo(algo) || !valid_prec(prec)) return 0;
    if (algo != NS_ALGO_FUSED && prec != NS_FP64) return 0;
    return layout(make_consts(p), algo, prec).total;
}

ns_status ns_set_fused_config(int32_t tile, int32_t zchunk)
{
    if (tile < -1 || tile >= TILE_COUNT || zchunk < 0) return NS_ERR_ARG;
    if (zchunk > 0 && zchunk < kMinZChunk) return NS_ERR_ARG;
    g_tile = tile;
    g_zchunk = zchunk;
    return NS_OK;
}

ns_status ns_set_fused_order(int32_t order)
{
    if (order != 0 && order != 1) return NS_ERR_ARG;
    g_order = order;
    return NS_OK;
}

int32_t ns_get_fused_order(void) { return g_order; }

ns_status ns_get_fused_config(const ns_params *p, ns_precision prec, int32_t *tile,
                              int32_t *zchunk)
{
    ns_status st = check_params(p);
    if (st != NS_OK) return st;
    if (!tile || !zchunk || !valid_prec(prec)) return NS_ERR_ARG;
    int t, z;
    choose_config(make_consts(p), prec, &t, &z);
    *tile = t;
    *zchunk = z;
    return NS_OK;
}

ns_status tgv_init(const ns_params *p, double *state, void *stream)
{
    ns_status st = check_params(p);
    if (st != NS_OK) return st;
    if (!state || !aligned(state, 16)) return NS_ERR_ARG;
    const Consts c = make_consts(p);
    NS_HIP_OK(launch_tgv_init(c, p, state, (hipStream_t)stream));
    return NS_OK;
}

ns_status ns_residual(const ns_params *p, ns_algo algo, const double *Q, double *R, void *work,
                      size_t work_bytes, void *stream)
{
    ns_status st = check_params(p);
    if (st != NS_OK) return st;
    if (!valid_algo(algo) || !Q || !R || !aligned(Q, 16) || !aligned(R, 16)) return NS_ERR_ARG;
    const Consts c = make_consts(p);
    const size_t n5b = 5 * (size_t)c.N * sizeof(double);
    if ((const char *)Q < (const char *)R + n5b && (const char *)R < (const char *)Q + n5b)
        return NS_ERR_ARG;   // overlap
    hipStream_t s = (hipStream_t)stream;
    if (algo == NS_ALGO_FUSED) {
        int tile, zc;
        choose_config(c, NS_FP64, &tile, &zc);
        const int order = g_order;
        if (!fused_order_supported(tile, order)) return NS_ERR_UNSUPPORTED;
        StageArgs a = {};
        a.order = order;
        a.qin = Q;
        a.rout = R;
        a.mode = 0;
        a.zchunk = zc;
        NS_HIP_OK(launch_fused_stage(c, a, NS_FP64, tile, s));
        return NS_OK;
    }
    const Layout L = layout(c, algo, NS_FP64);
    st = check_work(work, work_bytes, L.total);
    if (st != NS_OK) return st;
    if (algo == NS_ALGO_SOME) {
        NS_HIP_OK(rs_stage(c, Q, at<double>(work, L.G), nullptr, nullptr, nullptr, R, 0.0, 0.0, 0, s));
        return NS_OK;
    }
    NS_HIP_OK(stored_residual(c, Q, R, at<double>(work, L.stored), s));
    return NS_OK;
}

ns_status rk3_step(const ns_params *p, ns_algo algo, ns_precision prec, double dt, int32_t nsteps,
                   double *state, void *work, size_t work_bytes, ns_diag *diag_dev, void *stream)
{
    ns_status st = check_params(p);
    if (st != NS_OK) return st;
    if (!valid_algo(algo) || !valid_prec(prec) || !state || !aligned(state, 16)) return NS_ERR_ARG;
    if (diag_dev && !aligned(diag_dev, 8)) return NS_ERR_ARG;
    if (!std::isfinite(dt) || !(dt > 0.0) || nsteps < 0) return NS_ERR_ARG;
    if (algo != NS_ALGO_FUSED && prec != NS_FP64) return NS_ERR_UNSUPPORTED;
    const Consts c = make_consts(p);
    const Layout L = layout(c, algo, prec);
    st = check_work(work, work_bytes, L.total);
    if (st != NS_OK) return st;
    if (nsteps == 0) return NS_OK;
    hipStream_t s = (hipStream_t)stream;
    double *partial = at<double>(work, L.partial);
    double *acc = at<double>(work, L.acc);
    void *b1 = at<void>(work, L.b1);
    void *b2 = at<void>(work, L.b2);

    if (algo == NS_ALGO_FUSED) {
        FusedPlan f;
        st = make_fused_plan(p, prec, -1, 0, state, work, work_bytes, &f);
        if (st != NS_OK) return st;
        for (int32_t step = 0; step < nsteps; ++step)
            NS_HIP_OK(enqueue_fused_step(f, dt, diag_dev ? diag_dev + step : nullptr, s));
        return NS_OK;
    }

    if (algo == NS_ALGO_SOME) {
        double *G = at<double>(work, L.G);
        double *q1 = (double *)b1, *q2 = (double *)b2;
        for (int32_t step = 0; step < nsteps; ++step) {
            if (diag_dev) {
                NS_HIP_OK(launch_diag_partials(c, state, partial, s));
                NS_HIP_OK(launch_diag_finalize(c, partial, diag_num_blocks(c), diag_dev + step, s));
            }
            NS_HIP_OK(rs_stage(c, state, G, nullptr, acc, q1, nullptr, rk_a(0) * dt, rk_b(0) * dt, 1, s));
            NS_HIP_OK(rs_stage(c, q1, G, acc, acc, q2, nullptr, rk_a(1) * dt, rk_b(1) * dt, 2, s));
            NS_HIP_OK(rs_stage(c, q2, G, acc, nullptr, state, nullptr, rk_a(2) * dt, 0.0, 3, s));
        }
        return NS_OK;
    }

    // stored-derivative class
    double *R = at<double>(work, L.R);
    double *wk = at<double>(work, L.stored);
    double *q1 = (double *)b1, *q2 = (double *)b2;
    for (int32_t step = 0; step < nsteps; ++step) {
        if (diag_dev) {
            NS_HIP_OK(launch_diag_partials(c, state, partial, s));
            NS_HIP_OK(launch_diag_finalize(c, partial, diag_num_blocks(c), diag_dev + step, s));
        }
        NS_HIP_OK(stored_residual(c, state, R, wk, s));
        NS_HIP_OK(launch_rk_update(c, R, state, acc, q1, rk_a(0) * dt, rk_b(0) * dt, s));
        NS_HIP_OK(stored_residual(c, q1, R, wk, s));
        NS_HIP_OK(launch_rk_update(c, R, acc, acc, q2, rk_a(1) * dt, rk_b(1) * dt, s));
        NS_HIP_OK(stored_residual(c, q2, R, wk, s));
        NS_HIP_OK(launch_rk_update(c, R, acc, nullptr, state, rk_a(2) * dt, 0.0, s));
    }
    return NS_OK;
}

ns_status ns_stage_stream(const ns_params *p, int32_t stage, double *state, void *work,
                          size_t work_bytes, void *stream)
{
    ns_status st = check_params(p);
    if (st != NS_OK) return st;
    if (stage < 1 || stage > 3 || !state || !aligned(state, 16)) return NS_ERR_ARG;
    const Consts c = make_consts(p);
    const Layout L = layout(c, NS_ALGO_FUSED, NS_FP64);
    st = check_work(work, work_bytes, L.total);
    if (st != NS_OK) return st;
    double *acc = at<double>(work, L.acc);
    double *b1 = at<double>(work, L.b1), *b2 = at<double>(work, L.b2);
    const int64_t n5 = 5 * c.N;
    hipStream_t s = (hipStream_t)stream;
    if (stage == 1) NS_HIP_OK(launch_stream_stage(1, n5, state, nullptr, acc, b1, s));
    if (stage == 2) NS_HIP_OK(launch_stream_stage(2, n5, b1, acc, acc, b2, s));
    if (stage == 3) NS_HIP_OK(launch_stream_stage(3, n5, b2, acc, nullptr, state, s));
    return NS_OK;
}

ns_status diagnostics(const ns_params *p, const double *state, ns_diag *out_host, void *work,
                      size_t work_bytes, void *stream)
{
    ns_status st = check_params(p);
    if (st != NS_OK) return st;
    if (!state || !out_host || !aligned(state, 16)) return NS_ERR_ARG;
    const Consts c = make_consts(p);
    const Layout L = layout(c, NS_ALGO_FUSED, NS_FP64);
    st = check_work(work, work_bytes, diag_bytes(c));
    if (st != NS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    double *partial = at<double>(work, L.partial);
    ns_diag *rec = at<ns_diag>(work, L.rec);
    NS_HIP_OK(launch_diag_partials(c, state, partial, s));
    NS_HIP_OK(launch_diag_finalize(c, partial, diag_num_blocks(c), rec, s));
    NS_HIP_OK(hipMemcpyAsync(out_host, rec, sizeof(ns_diag), hipMemcpyDeviceToHost, s));
    NS_HIP_OK(hipStreamSynchronize(s));
    const double *v = (const double *)out_host;
    for (int k = 0; k < 8; ++k)
        if (!std::isfinite(v[k])) return NS_ERR_NONFINITE;
    return NS_OK;
}

}  // extern "C"
