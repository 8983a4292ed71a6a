/*
 * ns_tgv.h -- C ABI of the MI355X (gfx950) compressible Navier-Stokes
 * residual + low-storage RK3 library.
 *
 * Method: Jammy, Jacobs, Lusher & Sandham, "Energy efficiency of finite
 * difference algorithms on multicore CPUs, GPUs, and Intel Xeon Phi
 * processors" (arXiv:1709.09713):
 *   - governing equations: methodology section, mass / momentum / energy
 *     equations with skew-symmetric convection and Laplacian-form viscous
 *     terms, equation of state (pinprimitive) and (Tinprimitive);
 *   - spatial discretisation: fourth-order central stencils (fd), (sd),
 *     periodic in all three directions;
 *   - temporal discretisation: three-stage low-storage Runge-Kutta (rk3_tvd)
 *     arranged as in the generic-algorithm figure;
 *   - test case: the Taylor-Green vortex of the results section.
 *
 * Conventions for every entry point:
 *   - Fields are stored field-major: Q[v][k][j][i], v = 0..4 for
 *     (rho, rho*u0, rho*u1, rho*u2, rho*E), i (x) fastest.  A "state" is
 *     5*nx*ny*nz doubles in device memory.  Point (i,j,k) is at
 *     (i*hx, j*hy, k*hz), h = length / n.
 *   - Pointers named state, Q, R and work are DEVICE pointers owned by the
 *     caller (state, Q and R 16-byte aligned, else NS_ERR_ARG: the kernels
 *     load pairs of doubles; work 256-byte aligned; diag_dev 8-byte); the library keeps none of them after returning, except a
 *     batch, which keeps its members' state and work pointers until they
 *     are removed (ns_batch_add).  out_host is a host pointer.
 *   - stream is a hipStream_t (NULL = the default stream).  Calls are
 *     stream-ordered and asynchronous, except diagnostics(), which waits for
 *     its stream.
 *   - Arguments are validated before anything is enqueued; a failed
 *     validation returns an error and touches no memory.  HIP errors map to
 *     NS_ERR_DEVICE.  No C++ exception crosses this boundary.  The single-
 *     solve entry points allocate no device memory: scratch space is the
 *     caller's `work` buffer of at least ns_workspace_bytes() bytes
 *     (256-byte aligned).  A batch allocates its streams, events and
 *     diagnostics array once, in ns_batch_create.
 */
#ifndef NS_TGV_H
#define NS_TGV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NS_OK = 0,
    NS_ERR_ARG = -1,         /* null pointer, bad enum, non-finite or out-of-range scalar */
    NS_ERR_SHAPE = -2,       /* grid size outside [5, 2048] or too many points */
    NS_ERR_WORKSPACE = -3,   /* work_bytes smaller than ns_workspace_bytes() or misaligned */
    NS_ERR_DEVICE = -4,      /* a HIP call failed */
    NS_ERR_NONFINITE = -5,   /* diagnostics found a NaN or infinity */
    NS_ERR_NOMEM = -6,       /* a device or host allocation failed (batch creation only:
                                the single-solve calls allocate nothing) */
    NS_ERR_UNSUPPORTED = -7  /* valid but not provided (stored or intermediate-storage
                                class in FP32 storage) */
} ns_status;

/* The algorithm classes compared in the algorithms section.
 * NS_ALGO_STORED: every derivative is written to its own global array and
 *   the residual is assembled from those arrays (the baseline algorithm,
 *   BL).
 * NS_ALGO_FUSED: no derivative array; derivatives are evaluated on the fly
 *   from LDS-staged tiles and accumulated straight into the residual (the
 *   minimal-storage class RA / SN / SN2).
 * NS_ALGO_SOME: intermediate storage (RS / SS): only the nine
 *   velocity-gradient components du_i/dx_j are stored in global arrays each
 *   stage; every other derivative is evaluated inline, and the mixed
 *   viscous derivatives are first derivatives of the stored gradients. */
typedef enum { NS_ALGO_STORED = 0, NS_ALGO_FUSED = 1, NS_ALGO_SOME = 2 } ns_algo;

/* NS_FP64: all storage and arithmetic in double.
 * NS_FP32_STORE: the Runge-Kutta stage inputs are stored and differenced in
 *   float, as deviations from the uniform reference state (rho = 1,
 *   p = 1/(gamma M^2)); the RK accumulator, the state between steps and the
 *   diagnostic reductions stay double.  Fused class only. */
typedef enum { NS_FP64 = 0, NS_FP32_STORE = 1 } ns_precision;

/* Grid and non-dimensional parameters (methodology section; results
 * section: Re = 1600, Pr = 0.71, M = 0.1, gamma = 1.4, length = 2 pi).
 * n[d] in [5, 2048] with nx*ny*nz < 2^31; length[d] > 0; gamma > 1;
 * prandtl > 0; mach > 0; reynolds > 0 or +INFINITY (inviscid: 1/Re = 0 and
 * no heat conduction). */
typedef struct {
    int32_t n[3];
    double length[3];
    double gamma;
    double prandtl;
    double reynolds;
    double mach;
} ns_params;

/* Diagnostics of a state (the kinetic-energy / enstrophy quantities of the
 * validation data set named in the results section):
 *   mass = hx hy hz sum rho, momentum[i] = hx hy hz sum rho u_i,
 *   energy = hx hy hz sum rho E, kinetic_energy = mean(rho |u|^2 / 2),
 *   enstrophy = mean(rho |curl u|^2 / 2) with fourth-order first derivatives,
 *   dissipation = 2 enstrophy / Re. */
typedef struct {
    double mass;
    double momentum[3];
    double energy;
    double kinetic_energy;
    double enstrophy;
    double dissipation;
} ns_diag;

/* Human-readable name of a status code (static storage). */
const char *ns_status_string(ns_status s);

/* Bytes of one state (5 * nx*ny*nz doubles); 0 if params is invalid.
 * The state is double for both precisions. */
size_t ns_state_bytes(const ns_params *p);

/* Bytes of caller-provided scratch that ns_residual / rk3_step /
 * diagnostics need for this (algo, precision); 0 if the combination is
 * invalid or unsupported.  Pure function. */
size_t ns_workspace_bytes(const ns_params *p, ns_algo algo, ns_precision prec);

/* Write the Taylor-Green vortex initial state of the results section into
 * state (device, 5*N doubles):
 *   u0 = sin(x/L) cos(y/L) cos(z/L), u1 = -cos(x/L) sin(y/L) cos(z/L),
 *   u2 = 0, p = 1/(gamma M^2) + (cos(2x/L) + cos(2y/L))(2 + cos(2z/L))/16,
 *   rho = gamma M^2 p (T = 1), rho E = p/(gamma-1) + rho |u|^2 / 2,
 * with L = length[d] / (2 pi) per direction. */
ns_status tgv_init(const ns_params *p, double *state, void *stream);

/* One evaluation of the residual R(Q) (the right-hand sides of the mass,
 * momentum and energy equations, discretised with (fd)/(sd) and periodic
 * boundaries), FP64, with the chosen algorithm class.  Q and R are device
 * arrays of 5*N doubles and must not overlap; Q is not modified.  The
 * stored and intermediate-storage classes need work of
 * ns_workspace_bytes(p, algo, NS_FP64) bytes; the fused class keeps every
 * derivative on chip and uses no scratch, so with NS_ALGO_FUSED work and
 * work_bytes are ignored (NULL / 0 allowed). */
ns_status ns_residual(const ns_params *p, ns_algo algo, const double *Q,
                      double *R, void *work, size_t work_bytes, void *stream);

/* Advance state (device, 5*N doubles) in place by nsteps full steps of the
 * three-stage low-storage Runge-Kutta scheme: per step, with Q_acc = Q^n,
 * for k = 1..3: R = R(Q); Q = Q_acc + a_k dt R; Q_acc += b_k dt R, with
 * a = (2/3, 5/12, 3/5), b = (1/4, 3/20, 3/5).  dt > 0 and finite;
 * nsteps >= 0.  If diag_dev is not NULL it is a device array of nsteps
 * ns_diag records: record s receives the diagnostics of the state at the
 * start of step s (computed inside the first stage).  work needs
 * ns_workspace_bytes(p, algo, prec) bytes.  algo = NS_ALGO_STORED and
 * NS_ALGO_SOME require prec = NS_FP64 (else NS_ERR_UNSUPPORTED); their
 * per-step diagnostics take one extra pass over the state. */
ns_status rk3_step(const ns_params *p, ns_algo algo, ns_precision prec,
                   double dt, int32_t nsteps, double *state, void *work,
                   size_t work_bytes, ns_diag *diag_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rk3_step
 * of the fused class (NS_ALGO_FUSED, either precision, default launch shape
 * of the calling thread) with its workspace taken from a static device
 * array of ns_noalloc_scratch_bytes() bytes (64 MiB) that the library holds
 * on every GPU it runs on until the process ends, instead of a caller
 * buffer.  Enqueues exactly rk3_step's kernels; results are bit-identical to
 * rk3_step's.  Allocates nothing.  NS_ERR_WORKSPACE if
 * ns_workspace_bytes(p, NS_ALGO_FUSED, prec) exceeds that size (grids up to
 * about 80^3), checked before the device is touched; other errors as
 * rk3_step.  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (different streams or threads) race and must be
 * serialised by the caller. */
ns_status rk3_step_noalloc(const ns_params *p, ns_precision prec, double dt, int32_t nsteps,
                           double *state, ns_diag *diag_dev, void *stream);

/* Size in bytes of the static device workspace of rk3_step_noalloc. */
size_t ns_noalloc_scratch_bytes(void);

/* Diagnostics of state (device, 5*N doubles) into *out_host, in FP64 with a
 * fixed reduction order (bitwise reproducible).  Waits for stream.  work
 * needs ns_workspace_bytes(p, NS_ALGO_FUSED, NS_FP64) bytes.  Returns
 * NS_ERR_NONFINITE (after filling *out_host) if any value is not finite. */
ns_status diagnostics(const ns_params *p, const double *state,
                      ns_diag *out_host, void *work, size_t work_bytes,
                      void *stream);

/* Measurement support, not part of the method: move exactly the HBM bytes
 * of fused RK stage `stage` (1..3) in FP64 -- stage 1 reads state and writes
 * the next stage input and the accumulator, stage 2 reads both and writes
 * both, stage 3 reads both and writes state, the same buffers rk3_step uses
 * in work -- with a pointwise update instead of the residual.  Its rate is
 * the ceiling that the memory system allows the fused stage kernel's access
 * pattern.  work needs ns_workspace_bytes(p, NS_ALGO_FUSED, NS_FP64) bytes.
 * The update of every element, with a = 1/2, b = 1/4: stage 1 sets the
 * stage buffer to Q + a Q and the accumulator to Q + b Q; stage 2 sets the
 * second stage buffer to acc + a s1 and acc to acc + b s1; stage 3 sets
 * state to acc + a s2.  Stages 1, 2, 3 in a row thus leave 2.625 Q in state
 * (exact when the products and sums are).  NS_ERR_ARG for stage outside
 * 1..3. */
ns_status ns_stage_stream(const ns_params *p, int32_t stage, double *state, void *work,
                          size_t work_bytes, void *stream);

/* Launch shape of the fused kernel for later calls made by the calling
 * thread (each thread keeps its own setting; a batch member fixes its shape
 * when it is added).  tile selects the
 * (x, y) column tile of one block: 0 = 32x8, 1 = 16x16, 2 = 64x4,
 * 3 = 32x16, 4 = 16x8, 5 = 32x4, 6 = 16x4, 7 = 8x8 (threads = product, one
 * z column each); 8 = 16x8, 9 = 32x8, 10 = 16x4 with two threads per
 * column (one loads the planes and evaluates the momentum equations, the
 * other the mass and energy equations and the viscous terms); zchunk is the number of
 * z planes one block marches through (>= 1; 0 = automatic: the length that
 * minimises (rounds of device-resident blocks) x (planes each block
 * marches, chunk + 4 halo planes; + 5 for tiles 8-10)).  tile = -1
 * restores the automatic choice: tile 9 for NS_FP64, tile 0 for
 * NS_FP32_STORE.  For a given tile, residuals and states are bitwise
 * independent of zchunk (tiles 8-10 also of the tile among them); different tiles are separate compiled
 * instances and may differ at the rounding level (the compiler can contract
 * a multiply-add differently); per-step diagnostics also differ in the
 * order of their sums.
 * Returns NS_ERR_ARG for out-of-range values. */
ns_status ns_set_fused_config(int32_t tile, int32_t zchunk);

/* The (tile, zchunk) the fused kernel would use for p and prec in a call
 * made now by the calling thread. */
ns_status ns_get_fused_config(const ns_params *p, ns_precision prec,
                              int32_t *tile, int32_t *zchunk);

/* Evaluation order of the fused kernel's in-plane residual terms for later
 * calls of the calling thread (the SN / SN2 distinction of the
 * minimal-storage section):
 * 0 = grouped by equation, the momentum equations by velocity component
 * (default); 1 = grouped by derivative direction (all x derivatives of all
 * equations, then all y derivatives).  The two orders sum the same terms
 * with a different association, so results differ at the rounding level
 * only.  Order 1 is compiled for tiles 4 (16x8) and 0 (32x8) only: rk3_step,
 * ns_residual and ns_batch_add return NS_ERR_UNSUPPORTED for it with any
 * other tile.  NS_ERR_ARG for other values. */
ns_status ns_set_fused_order(int32_t order);

/* The calling thread's evaluation order (0 or 1). */
int32_t ns_get_fused_order(void);

/* ------------------------------------------------------------------------
 * Batched execution: many independent solves (different grid sizes,
 * Reynolds and Mach numbers, time steps, step budgets) advanced together.
 * Each member runs exactly the launches of rk3_step with the fused class
 * (residual of the governing-equations section, RK3 of the time-advancement
 * section) under its own launch shape; a batch step queues one RK3 step of
 * every member with steps left (largest grids first), members spread over
 * up to 8 internal HIP streams (balanced by grid points) that fork from and
 * join back into the caller's stream, so small grids overlap on the device.
 * With the caller's stream that is up to 5 streams: on a device with 4
 * hardware queues per process, 3 internal streams measured fastest.  Per-point
 * arithmetic never depends on the other members: a solve gives identical
 * bits alone and in any mix.  Solves join (ns_batch_add) and leave
 * (ns_batch_remove) between steps while the others keep their state.
 * Ownership: the batch owns its streams, events and (with diagnostics) a
 * device array of one ns_diag per slot; states and workspaces stay
 * caller-owned, must outlive their membership, and may not be shared
 * between members.  Calls on one batch are not thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct ns_batch ns_batch;

typedef struct {
    ns_params p;        /* grid and physics of this solve */
    double dt;          /* > 0, finite */
    int32_t steps;      /* RK3 steps to run (>= 0) */
    int32_t tile;       /* launch tile as in ns_set_fused_config, -1 = default */
    int32_t zchunk;     /* z planes per block (>= 1), 0 = default */
    double *state;      /* device, 5*N doubles: initial state in, result out */
    void *work;         /* device, >= ns_workspace_bytes(p, NS_ALGO_FUSED, batch
                           precision) bytes, 256-byte aligned */
    size_t work_bytes;
} ns_instance;

/* Create a batch with room for max_instances (1..4096) solves advanced in
 * precision prec over nstreams (1..8) internal streams; with_diagnostics
 * != 0 computes each member's diagnostics of the state at the start of
 * every step it runs (last one readable with ns_batch_poll).  Allocates
 * streams, events and the diagnostics array (NS_ERR_NOMEM if an allocation
 * runs out of memory, NS_ERR_DEVICE for other HIP failures); NS_ERR_ARG for
 * bad arguments. */
ns_status ns_batch_create(int32_t max_instances, ns_precision prec,
                          int32_t nstreams, int32_t with_diagnostics,
                          ns_batch **out);

/* Wait for the batch's streams and free what the batch owns.  Caller
 * buffers are untouched. */
ns_status ns_batch_destroy(ns_batch *b);

/* Admit a solve into a free slot (*slot).  It runs its `steps` steps during
 * later ns_batch_step calls, in stream order after work queued before them
 * on their stream (so a tgv_init queued there first is seen).  Host-side
 * only.  NS_ERR_ARG / NS_ERR_SHAPE / NS_ERR_WORKSPACE as rk3_step for the
 * instance, NS_ERR_ARG if its buffers overlap each other or another
 * member's, NS_ERR_WORKSPACE if no slot is free. */
ns_status ns_batch_add(ns_batch *b, const ns_instance *inst, int32_t *slot);

/* Retire a slot (finished or not).  Host-side only: its state holds the
 * last step queued, once the caller's stream of the last ns_batch_step has
 * reached that point. */
ns_status ns_batch_remove(ns_batch *b, int32_t slot);

/* Queue nsteps RK3 steps of every member with steps left (a member stops at
 * its own budget), ordered after earlier work on `stream`; later work on
 * `stream` sees the results.  Asynchronous. */
ns_status ns_batch_step(ns_batch *b, int32_t nsteps, void *stream);

/* Run later ns_batch_step calls through HIP graphs (enable = 1) or eagerly
 * (0, the default).  With graphs, 8 batch steps of the members that have
 * steps left are captured once into a graph on a batch-owned stream, and
 * the graph is replayed while that set of members stays the same; adding,
 * removing or a member running out of steps triggers a new capture, and
 * steps that do not fill a whole graph run eagerly.  The launches are the
 * eager ones, so results are bit-identical.  The first enable creates a
 * stream and two events (NS_ERR_DEVICE on failure); NS_ERR_ARG for other
 * values of enable.  A failed capture or replay makes ns_batch_step return
 * NS_ERR_DEVICE. */
ns_status ns_batch_set_graphs(ns_batch *b, int32_t enable);

/* Fill host arrays of max_instances entries (any may be NULL) with each
 * slot's steps left (-1 for a free slot) and steps queued so far; with
 * diag non-NULL (batch created with diagnostics, else NS_ERR_ARG) copy the
 * diagnostics array and synchronise `stream`. */
ns_status ns_batch_poll(ns_batch *b, int32_t *steps_left, int32_t *steps_done,
                        ns_diag *diag, void *stream);

/* Capacity, occupied slots and internal stream count. */
ns_status ns_batch_info(const ns_batch *b, int32_t *max_instances,
                        int32_t *active, int32_t *nstreams);

#ifdef __cplusplus
}
#endif

#endif /* NS_TGV_H */
