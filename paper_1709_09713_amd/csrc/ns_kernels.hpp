// ns_kernels.hpp -- launch interfaces of the device kernels (host side).
#pragma once

#include "ns_common.hpp"

namespace ns {

// Column-tile shapes of the fused kernel.  Tiles 0-7: threads = BX * BY,
// one z column each (ns_fused.hip).  Tiles 8-10 (_2G): 2 * BX * BY
// threads, two per column: the momentum equations in one wave group, the
// mass and energy equations and the viscous terms in the other
// (ns_split.hip).  Chosen per problem by the
// autotuner or by the default rule.
enum {
    TILE_32x8 = 0, TILE_16x16 = 1, TILE_64x4 = 2, TILE_32x16 = 3,
    TILE_16x8 = 4, TILE_32x4 = 5, TILE_16x4 = 6, TILE_8x8 = 7,
    TILE_16x8_2G = 8, TILE_32x8_2G = 9, TILE_16x4_2G = 10, TILE_COUNT = 11
};

// One fused launch: residual only (mode 0) or RK stage 1..3.
struct StageArgs {
    const void *qin;        // stencil input state (double, or float deviations)
    const double *acc_in;   // RK accumulator in (stages 2, 3)
    double *acc_out;        // RK accumulator out (stages 1, 2)
    void *qout;             // stage output (stages 1, 2: next stage input; 3: state)
    double *rout;           // residual output (mode 0)
    double a_dt, b_dt;      // a_k dt and b_k dt
    int mode;               // 0 = residual, 1..3 = RK stage
    int zchunk;             // planes per block along z
    double *diag_partial;   // per-block diagnostic partial sums, or nullptr
    int order;              // in-plane evaluation order: 0 by equation, 1 by direction
};

void tile_dims(int tile, int *bx, int *by);
int64_t fused_num_blocks(const Consts &c, int tile, int zchunk);
bool fused_order_supported(int tile, int order);
// Stage-kernel blocks resident on the current device at once (0 if the
// device cannot be queried).
int fused_resident_blocks(ns_precision prec, int tile);
hipError_t launch_fused_stage(const Consts &c, const StageArgs &s, ns_precision prec,
                              int tile, hipStream_t st);
// The two-group kernel (tiles 8-10): stage launch and resident blocks.
bool split_tile(int tile);
int split_resident_blocks(ns_precision prec, int tile);
hipError_t launch_split_stage(const Consts &c, const StageArgs &s, ns_precision prec, int tile,
                              hipStream_t st);
// Planes a block marches beyond its chunk (halo and pipeline depth).
int fused_extra_planes(int tile);

// Argument check of an ns_params (grid range, finite positive lengths and
// physics); NS_OK, NS_ERR_ARG or NS_ERR_SHAPE.
ns_status validate_params(const ns_params *p);

// A validated fused-class RK3 plan for one solve: constants, launch shape
// and the carve-up of its workspace.  rk3_step and the batch scheduler
// enqueue steps through it, so both run the same launches.
struct FusedPlan {
    Consts c;
    ns_precision prec;
    int tile, zchunk, order;
    int64_t nblk;
    double *state, *partial, *acc;
    void *b1, *b2;
};
// tile -1 / zchunk 0 take the process-wide or default launch shape.
// Validates everything (params, precision, shape, workspace) first.
ns_status make_fused_plan(const ns_params *p, ns_precision prec, int tile, int zchunk,
                          double *state, void *work, size_t work_bytes, FusedPlan *out);
hipError_t enqueue_fused_step(const FusedPlan &f, double dt, ns_diag *diag_out, hipStream_t s);

// Diagnostics: per-block partial sums of a state, then a one-block fixed-order
// final reduction into an ns_diag record.
int64_t diag_num_blocks(const Consts &c);
hipError_t launch_diag_partials(const Consts &c, const double *state, double *partial,
                                hipStream_t st);
hipError_t launch_diag_finalize(const Consts &c, const double *partial, int64_t nblocks,
                                ns_diag *out, hipStream_t st);

// The bytes of one fused FP64 RK stage (1..3) over the same buffers, with
// a pointwise update instead of the residual (the achievable ceiling of the
// stage kernel's memory traffic).  n5 = number of doubles in a field set.
hipError_t launch_stream_stage(int stage, int64_t n5, const double *qin, const double *acc_in,
                               double *acc_out, double *qout, hipStream_t st);

// Taylor-Green initial state.
hipError_t launch_tgv_init(const Consts &c, const ns_params *p, double *state, hipStream_t st);

// Stored-derivative (baseline) class.
size_t stored_workspace_doubles(const Consts &c);
// Intermediate-storage class: nine gradient arrays; one stage = gradient
// sweep + residual/RK sweep (mode 0 writes R to rout).
size_t rs_workspace_doubles(const Consts &c);
hipError_t rs_stage(const Consts &c, const double *qin, double *G, const double *acc_in,
                    double *acc_out, double *qout, double *rout, double a_dt, double b_dt,
                    int mode, hipStream_t st);
hipError_t stored_residual(const Consts &c, const double *Q, double *R, double *work,
                           hipStream_t st);
hipError_t launch_rk_update(const Consts &c, const double *R, const double *acc_in,
                            double *acc_out, double *qout, double a_dt, double b_dt,
                            hipStream_t st);

}  // namespace ns
