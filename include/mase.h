/*
 * mase.h -- C ABI of the MI355X multi-area WLS state-estimation library.
 *
 * The library implements the per-Gauss-Newton-iteration pipeline of
 * hierarchical multi-area state estimation with boundary condensation
 * (arXiv 2604.23175, Sections 2-4):
 *
 *   1. measurement evaluation fused with direct accumulation of each area's
 *      normal-equation blocks G^k = H_k^T W_k H_k and b^k = H_k^T W_k r_k
 *      (Eq. 4 and Eq. 7, Section 4.2), without forming H;
 *   2. per-area elimination of the internal variables: a sparse Cholesky
 *      factorisation of G_ii^k that leaves the dense Schur block
 *      S_b^k = G_bb - G_bi G_ii^-1 G_ib and the condensed right-hand side
 *      bhat_b^k (Eq. 8-10, Section 4.3);
 *   3. assembly of the boundary system S_Gamma = sum_k E_k^T S_b^k E_k,
 *      bhat_Gamma = sum_k E_k^T bhat_b^k (Eq. 11, Section 4.4), its Cholesky
 *      solve, scatter-back dx_b^k = E_k dx_Gamma and interior recovery
 *      dx_i^k = G_ii^-1 (b_i - G_ib dx_b^k) (Eq. 8), then x += dx.
 *
 * Many measurement snapshots of one grid are processed together (all areas
 * and all snapshots in one launch per stage).
 *
 * Conventions
 * -----------
 * - State: bus voltage angle theta (rad) and magnitude |V| (p.u.).  The
 *   slack bus angle is the reference, fixed at 0, and is not a state
 *   variable (n = 2N - 1, Section 5.2 counts 5737 = 2*2869 - 1 states).
 * - Branch model: pi model, series impedance r + jx, total line charging b
 *   split b/2 per end, no taps, no bus shunts.
 * - Measurements (Eq. 4, types below): |V| at a bus, active/reactive injection
 *   at a bus, active/reactive flow at the from end or the to end of a branch.
 *   Weights default to w_i = 1/sigma_i^2 (W = R^-1, Eq. 2); a zero weight
 *   masks a row without changing any structure (Section 4.1).
 * - Measurement ownership: |V| and injections at bus i belong to area(i); a
 *   from-end flow to area(from), a to-end flow to area(to).  Boundary buses
 *   are the terminals of branches whose ends lie in different areas; area
 *   k's local boundary set is its own boundary buses plus the foreign
 *   terminal of each of its cut branches (Section 2.3).
 * - Canonical orders used by every export: the global variable id of bus b
 *   is 2b for theta (never for the slack) and 2b+1 for |V|; an area's local
 *   variables are its internal buses then its local boundary buses, each in
 *   increasing bus id, theta before |V|; Gamma lists all boundary buses in
 *   increasing bus id, theta before |V|.
 * - Memory: every pointer argument is caller-owned.  Host pointers are read
 *   (or written) only during the call; `mase_create` copies what it needs.
 *   Pointers named *_dev are device pointers on the context's stream.
 * - Errors: 0 is success, negative values are errors (MASE_ERR_*), and
 *   `mase_solve` returns MASE_NOT_CONVERGED (+1) when a snapshot reached
 *   max_iter.  `mase_last_error` returns a message for the last failure.
 * - Threading: a context is used by one host thread at a time.
 */
#ifndef MASE_H
#define MASE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mase_ctx mase_ctx;

/* Measurement types (Eq. 4: one template per type). */
enum {
  MASE_VM = 0,   /* |V| at bus meas_at */
  MASE_PINJ = 1, /* active injection at bus meas_at */
  MASE_QINJ = 2, /* reactive injection at bus meas_at */
  MASE_PF = 3,   /* active flow at the from end of branch meas_at */
  MASE_QF = 4,   /* reactive flow at the from end of branch meas_at */
  MASE_PT = 5,   /* active flow at the to end of branch meas_at */
  MASE_QT = 6    /* reactive flow at the to end of branch meas_at */
};

/* Return codes. */
enum {
  MASE_OK = 0,
  MASE_NOT_CONVERGED = 1,
  MASE_ERR_ARG = -1,        /* bad argument: index out of range, sigma <= 0,
                               non-finite value, area without internal bus,
                               disconnected area, size over a limit */
  MASE_ERR_STATE = -2,      /* call out of order (e.g. no measurements set) */
  MASE_ERR_NOT_POSDEF = -3, /* a non-positive pivot in G_ii^k or S_Gamma:
                               the area or boundary system is unobservable */
  MASE_ERR_HIP = -4,        /* a HIP runtime call failed */
  MASE_ERR_OOM = -5,        /* device or host allocation failed */
  MASE_ERR_NO_DEVICE = -6   /* a GPU call on a host-only context */
};

/* How the boundary system S_Gamma dx_Gamma = bhat_Gamma is factored. */
enum {
  MASE_GAMMA_SPARSE = 0, /* minimum-degree ordering of Gamma, sparse
                            elimination of all but the root separator, dense
                            Cholesky of that separator block (default) */
  MASE_GAMMA_DENSE = 1   /* dense Cholesky of the whole S_Gamma */
};

typedef struct {
  void* stream;          /* hipStream_t to run on; NULL = library-owned stream */
  int32_t batched;       /* 1 (default): one launch per stage over all areas x
                            snapshots.  0: the paper's plain schedule -- one
                            snapshot at a time, per-area launches on per-area
                            streams, no graph */
  int32_t use_graph;     /* 1: capture one GN iteration as a hipGraph and
                            replay it (batched mode only); default 1 */
  int32_t gamma_mode;    /* MASE_GAMMA_SPARSE (default) or MASE_GAMMA_DENSE */
  int32_t host_only;     /* 1: build the maps and symbolic structures only,
                            touch no GPU (exports work, solves return
                            MASE_ERR_NO_DEVICE) */
  int32_t autotune;      /* 1: the first mase_solve times the candidate
                            schedules (pipeline groups 1/2/4/8, supernodal or
                            level-scheduled boundary elimination, the dense
                            block's panel width, then the LDS elimination's
                            workgroup size) for two GN iterations on the
                            current measurements, keeps the fastest and
                            restores the state; results are then the chosen
                            schedule's (bitwise the same for every choice) */
  const char* tune_cache;/* path of a text file caching that choice per grid
                            structure, batch size and device (read before
                            tuning, appended after), or NULL */
  int32_t local_steps;    /* Gauss-Newton steps of every area's local problem
                            with its boundary held (Eq. 6) before each
                            condensed step: re-assembly, elimination and
                            back substitution with dx_b = 0, internal
                            variables only.  Default 0 (every iteration is
                            one exact GN step); batched mode only */
  int32_t pipeline_groups;/* mase_solve in the batched graph mode: split the
                            snapshots into this many groups that iterate on
                            their own streams, so that one group's boundary
                            solve (latency-bound, few CUs) overlaps the next
                            group's area stages.  0 (default) or 1: off;
                            the autotuner also tries 2, 4 and 8.  Results
                            are bitwise identical for every value */
} mase_options;

/* Fill `opt` with the defaults listed above. */
void mase_default_options(mase_options* opt);

/*
 * Build a context for one grid topology, partition and measurement set, for
 * up to n_snap snapshots processed together (Sections 2.3, 4.1, 5.1: all
 * templates, maps and buffers are built once and stay on the device).
 *
 *   br_from, br_to [n_branch]   bus indices in [0, n_bus), from != to
 *   br_r, br_x, br_b [n_branch] series r, x (r + jx != 0) and total charging
 *   slack_bus                   reference bus (angle 0)
 *   bus_area [n_bus]            area index in [0, n_area) of every bus; each
 *                               area must be connected and own at least one
 *                               internal (non-boundary) bus
 *   meas_type, meas_at [n_meas] type (MASE_VM..MASE_QT) and bus/branch index
 *   meas_sigma [n_meas]         standard deviation, > 0
 *   n_snap                      snapshots per batch, >= 1
 *   opt                         options or NULL for defaults
 *
 * On success *out receives the context.  Fails with MASE_ERR_ARG on invalid
 * input, MASE_ERR_OOM / MASE_ERR_HIP on device trouble.
 */
int mase_create(int32_t n_bus, int32_t n_branch,
                const int32_t* br_from, const int32_t* br_to,
                const double* br_r, const double* br_x, const double* br_b,
                int32_t slack_bus, int32_t n_area, const int32_t* bus_area,
                int32_t n_meas, const int32_t* meas_type, const int32_t* meas_at,
                const double* meas_sigma, int32_t n_snap,
                const mase_options* opt, mase_ctx** out);

void mase_destroy(mase_ctx* ctx);

/* Message describing the last error on this thread (never NULL). */
const char* mase_last_error(void);

/* Short name of a return code. */
const char* mase_strerror(int code);

/*
 * Measurements z [n_snap][n_meas] (host) and weights w [n_meas] (host, or
 * NULL for 1/sigma^2; w = 0 masks a row, Section 4.1).  Copied to the device.
 */
int mase_set_measurements(mase_ctx* ctx, const double* z, const double* w);

/* Same with device pointers (w_dev NULL: 1/sigma^2); both are copied on the
 * context's stream, so the caller's buffers must stay valid until that
 * stream reaches the copy. */
int mase_set_measurements_dev(mase_ctx* ctx, const double* z_dev, const double* w_dev);

/*
 * Starting state vm, va [n_snap][n_bus] (host), or NULL for flat start
 * (|V| = 1, theta = 0).  The slack angle is forced to 0.  Marks every
 * snapshot active and clears the iteration counters.
 */
int mase_set_state(mase_ctx* ctx, const double* vm, const double* va);
int mase_set_state_dev(mase_ctx* ctx, const double* vm_dev, const double* va_dev);

/*
 * One Gauss-Newton iteration (Eq. 3 solved through Eq. 7-11) for every
 * active snapshot: assembly, local condensation, boundary assembly and
 * solve, scatter-back, interior recovery, x += dx.  max_abs_dx [n_snap]
 * (host, may be NULL) receives max_i |dx_i| of each snapshot (0 for frozen
 * snapshots).  Snapshots whose step is below the tolerance of the last
 * mase_solve (default 1e-6) are frozen afterwards.  A snapshot that hits a
 * non-positive pivot is frozen without an update; the others are updated,
 * max_abs_dx is written, and the call returns MASE_ERR_NOT_POSDEF.
 */
int mase_gn_iter(mase_ctx* ctx, double* max_abs_dx);

/*
 * Iterate until every snapshot has taken a step with max |dx| < tol, or
 * max_iter iterations (the paper caps Gauss-Newton at 10, Section 5.1).
 * iters [n_snap] and converged [n_snap] (host, may be NULL) receive the
 * per-snapshot step count and flag.  Returns MASE_NOT_CONVERGED if any
 * snapshot did not converge.  A snapshot whose G_ii^k or S_Gamma has a
 * non-positive pivot is frozen at the state before that iteration (its
 * converged flag is 0) while the others iterate on; the call then returns
 * MASE_ERR_NOT_POSDEF with iters and converged written for every snapshot.
 */
int mase_solve(mase_ctx* ctx, double tol, int32_t max_iter, int32_t* iters,
               int32_t* converged);

/*
 * Continuous batching over a stream of n_total snapshots (each solved as in
 * mase_solve: Gauss-Newton, Eq. 3 through Eq. 7-11, until a step has
 * max |dx| < tol, at most max_iter steps).  The context's n_snap snapshots
 * act as slots: after every batched iteration, a slot whose snapshot has
 * converged, failed or used max_iter steps writes that snapshot's state to
 * the outputs and takes the next snapshot of the stream, so no iteration is
 * spent on a batch in which only a few snapshots are still running.  Each
 * snapshot's arithmetic is that of mase_solve (results are bitwise equal to
 * solving it in a batch from the same start).
 *
 *   z_dev        [n_total][n_meas] measurements (device); weights are those
 *                of the last mase_set_measurements call, else 1/sigma^2
 *   vm0_dev,
 *   va0_dev      [n_total][n_bus] starting states (device), or both NULL for
 *                flat start; the slack angle is forced to 0
 *   vm_dev,
 *   va_dev       [n_total][n_bus] solved states (device, written)
 *   iters,
 *   converged    [n_total] (host, may be NULL) per-snapshot step count and
 *                flag
 *
 * The caller's buffers must stay valid until the call returns (it
 * synchronises the context's stream).  Needs the batched schedule
 * (MASE_ERR_ARG otherwise), 0 <= n_total <= 2^30.  Runs the autotuner first
 * when the context asks for it and has not tuned yet.  Returns
 * MASE_NOT_CONVERGED if any snapshot did not converge, MASE_ERR_NOT_POSDEF
 * (outputs still written) if any hit a non-positive pivot.  Afterwards every
 * slot is frozen; the slots' measurements and states are those of the last
 * snapshots that passed through them.
 */
int mase_solve_stream(mase_ctx* ctx, const double* z_dev, const double* vm0_dev, const double* va0_dev,
                      int64_t n_total, double tol, int32_t max_iter, double* vm_dev, double* va_dev,
                      int32_t* iters, int32_t* converged);

/*
 * mase_solve_stream with host buffers at both ends, the solve timed end to
 * end as in Section 5.1 (measurements in, states out): z_host
 * [n_total][n_meas] is uploaded in chunks of n_snap snapshots on a copy
 * stream (default priority) ahead of the stream position, so the copies
 * overlap the iterations of earlier snapshots, and the solved states go to
 * vm_host, va_host [n_total][n_bus] chunk by chunk as soon as every snapshot
 * of a chunk has left its slot.  vm0_host, va0_host [n_total][n_bus]: starting
 * states, or both NULL for flat start.  Host buffers should be pinned
 * (hipHostMalloc) for the copies to overlap; pageable memory is correct but
 * serialises them.  work_dev: caller-owned device workspace of work_len
 * doubles, at least mase_stream_host_work(ctx, n_total, vm0_host != NULL),
 * that holds the device copies of z, the starting states and the results.
 * iters, converged, arguments, return codes and results as in
 * mase_solve_stream (bitwise equal states).  Host buffers must stay valid
 * until the call returns.
 */
int mase_solve_stream_host(mase_ctx* ctx, const double* z_host, const double* vm0_host, const double* va0_host,
                           int64_t n_total, double tol, int32_t max_iter, double* vm_host, double* va_host,
                           int32_t* iters, int32_t* converged, double* work_dev, int64_t work_len);

/*
 * mase_solve_stream for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, results (bitwise) and return codes, but the
 * stream's bookkeeping (slot tables and per-snapshot results) lives in a
 * fixed 4 MiB device array of the library instead of context allocations,
 * and nothing is allocated: no autotuning, and when the context has no
 * instantiated iteration graph yet the kernels are launched directly.
 * Limit: 3 n_snap + 2 + 2 n_total <= 2^20 ints, i.e. n_total at most
 * mase_stream_noalloc_max(ctx); larger n_total returns MASE_ERR_ARG before
 * any device work.  Every no-alloc call on one GPU shares that array (one
 * copy per GPU, held until the process ends), so calls that overlap on one
 * GPU, from any context or thread, race and must be serialised by the
 * caller.
 */
int mase_solve_stream_noalloc(mase_ctx* ctx, const double* z_dev, const double* vm0_dev, const double* va0_dev,
                              int64_t n_total, double tol, int32_t max_iter, double* vm_dev, double* va_dev,
                              int32_t* iters, int32_t* converged);

/* Largest n_total mase_solve_stream_noalloc accepts for this context; -1 on
 * a null context. */
int64_t mase_stream_noalloc_max(const mase_ctx* ctx);

/* Doubles of device workspace mase_solve_stream_host needs for n_total
 * snapshots (with_start != 0: starting states given); -1 on a bad argument. */
int64_t mase_stream_host_work(const mase_ctx* ctx, int64_t n_total, int32_t with_start);

/* Current state vm, va [n_snap][n_bus] (host / device). */
int mase_state(mase_ctx* ctx, double* vm, double* va);
int mase_state_dev(mase_ctx* ctx, double* vm_dev, double* va_dev);

/* WLS objective J = r^T W r (Eq. 2) at the current state, J [n_snap] (host). */
int mase_objective(mase_ctx* ctx, double* J);

/*
 * Measurement functions h(x) at states vm, va [n_snap][n_bus] (device) into
 * h_dev [n_snap][n_meas] (device): the per-type templates of Eq. 4 in
 * evaluation-only mode.  Does not change the context's state.
 */
int mase_eval_h_dev(mase_ctx* ctx, const double* vm_dev, const double* va_dev, double* h_dev);

/* ---- learned warm start (an extension of the paper's method) ----
 *
 * One MLP per area maps the area's measurements, normalised as
 * (z - z_mean) / sigma, through two ReLU hidden layers of `hidden` units to
 * a starting (|V|, theta) for each of the area's own buses (outputs
 * standardised by y_mean / y_std).  Weights are bfloat16 copies of FP32
 * master weights; products run on bf16 MFMA with FP32 accumulation; Adam
 * updates the masters.  Gauss-Newton in FP64 has the last word: a prediction
 * is used for a snapshot only if its objective J (Eq. 2) is not worse than
 * that of the flat start.
 *
 * Parameter vector (FP32, host order for set/get): for each area in order,
 * W1 [m_k x hidden], b1 [hidden], W2 [hidden x hidden], b2 [hidden],
 * W3 [hidden x o_k], b3 [o_k], row-major ("inputs x outputs").  The inputs of
 * area k are its measurements and its outputs are the global variable ids of
 * its own buses (2*bus theta, 2*bus+1 |V|; the slack angle is an output
 * whose prediction is replaced by 0), both in the order mase_mlp_io_map
 * returns.
 */
typedef struct mase_mlp mase_mlp;

/* Allocate the per-area networks of `ctx` (device), zero-initialised; up to
 * max_batch samples per training step (and at least n_snap). */
int mase_mlp_create(mase_ctx* ctx, int32_t hidden, int32_t max_batch, mase_mlp** out);
void mase_mlp_destroy(mase_mlp* mlp);

/* Sizes: area >= 0 gives that area's input and output counts, area = -1 the
 * totals; n_param is the length of the parameter vector. */
int mase_mlp_info(const mase_mlp* mlp, int32_t area, int32_t* n_in, int32_t* n_out, int64_t* n_param);

/* Area k's input measurement ids [n_in] and output variable ids [n_out]. */
int mase_mlp_io_map(const mase_mlp* mlp, int32_t area, int32_t* in_meas, int32_t* out_var);

/* Parameters (host FP32, n_param); set also clears the Adam moments. */
int mase_mlp_set_params(mase_mlp* mlp, const float* params);
int mase_mlp_get_params(mase_mlp* mlp, float* params);

/* Normalisation: z_mean [n_meas]; y_mean, y_std [2 n_bus] by variable id. */
int mase_mlp_set_norm(mase_mlp* mlp, const double* z_mean, const double* y_mean, const double* y_std);

/*
 * Normalisation from a training set of n snapshots (device, row-major):
 * z_dev [n][n_meas] measurements, vm_dev, va_dev [n][n_bus] their solved
 * states.  Sets z_mean to the per-measurement mean of z, y_mean / y_std to
 * the per-variable mean and sample standard deviation (denominator n - 1,
 * replaced by 1 where it is at most 1e-6) of the outputs, interleaved per bus
 * as (theta, |V|), all computed on the device in fixed order.  in_rms
 * [n_area] (host, may be NULL) receives, per area, the RMS over the area's
 * inputs and the n snapshots of the normalised input (z - z_mean) / sigma
 * (used to scale the first layer's initial weights).  n >= 1.
 */
int mase_mlp_fit_norm(mase_mlp* mlp, const double* z_dev, const double* vm_dev, const double* va_dev, int32_t n,
                      double* in_rms);

/* The normalisation in use: z_mean [n_meas], y_mean, y_std [2 n_bus] (host);
 * MASE_ERR_STATE if none was set. */
int mase_mlp_get_norm(const mase_mlp* mlp, double* z_mean, double* y_mean, double* y_std);

/* Mean squared error of the standardised outputs over a batch of
 * measurements z_dev [batch][n_meas] against states vm_dev, va_dev
 * [batch][n_bus] (device), and its gradient (host FP32 [n_param], may be
 * NULL).  No update. */
int mase_mlp_loss_grad(mase_mlp* mlp, const double* z_dev, const double* vm_dev, const double* va_dev,
                       int32_t batch, double* loss, float* grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the same loss; loss
 * (host, may be NULL) receives the loss before the step. */
int mase_mlp_train_step(mase_mlp* mlp, const double* z_dev, const double* vm_dev, const double* va_dev,
                        int32_t batch, float lr, double* loss);

/* Predicted states vm_dev, va_dev [batch][n_bus] (device) for z_dev. */
int mase_mlp_predict_dev(mase_mlp* mlp, const double* z_dev, int32_t batch, double* vm_dev, double* va_dev);

/*
 * Warm start for the context's current measurements: predict every
 * snapshot's state, evaluate J at the prediction and at flat start, keep the
 * prediction where J(pred) <= J(flat) and flat start elsewhere; accepted
 * [n_snap] (host, may be NULL) receives 1 where the prediction was kept.
 * Marks every snapshot active, as mase_set_state does.
 */
int mase_warm_start(mase_ctx* ctx, mase_mlp* mlp, int32_t* accepted);

/* Acceptance cap of mase_warm_start: a prediction is kept only if, besides
 * J(pred) <= J(flat), also J(pred) <= j_cap.  Default +inf (the objective
 * comparison alone).  A caller calibrates it on held-out snapshots when
 * predictions that beat flat start on J still cost Gauss-Newton iterations.
 * Since J >= 0, a negative cap rejects every prediction, and mase_warm_start
 * then sets flat start without evaluating the network or the objectives
 * (mase_warm_start_objectives reports NaN).  j_cap must not be NaN
 * (MASE_ERR_ARG). */
int mase_mlp_set_accept_cap(mase_mlp* mlp, double j_cap);

/* J(pred) and J(flat) of every snapshot [n_snap] (host) as evaluated by the
 * last mase_warm_start; MASE_ERR_STATE before the first call. */
int mase_warm_start_objectives(const mase_mlp* mlp, double* j_pred, double* j_flat);

/* ---- per-stage timing ---- */

/* Kernel stages of one iteration, in launch order. */
enum {
  MASE_STAGE_ASSEMBLE = 0,   /* fused evaluation + accumulation (Eq. 7) */
  MASE_STAGE_CONDENSE,       /* per-area elimination (Eq. 8-10) */
  MASE_STAGE_GAMMA_GATHER,   /* boundary assembly (Eq. 11) */
  MASE_STAGE_GAMMA_SPARSE,   /* sparse elimination inside the boundary system */
  MASE_STAGE_GAMMA_DENSE,    /* dense Cholesky + solve of its trailing block */
  MASE_STAGE_GAMMA_BACK,     /* back substitution inside the boundary system */
  MASE_STAGE_BACKSOLVE,      /* scatter-back + interior recovery (Eq. 8) */
  MASE_STAGE_UPDATE,         /* x += dx, convergence */
  MASE_STAGE_LOCAL,          /* all kernels of the local steps (mase_options.local_steps) */
  MASE_N_STAGE
};

/*
 * enable != 0: record a pair of HIP events on the context's stream around
 * every stage kernel of the batched schedule and accumulate their elapsed
 * times after each iteration; clears the accumulators.  While enabled, the
 * batched schedule launches its kernels directly instead of replaying the
 * captured graph (event pairs inside a graph cannot be timed).  enable == 0
 * stops recording and returns to graph replay.
 */
int mase_profile(mase_ctx* ctx, int32_t enable);

/*
 * Accumulated per-stage kernel time in ms, launch counts and work units (the
 * number of active snapshots each launch processed), each [MASE_N_STAGE]
 * (host, any may be NULL).
 */
int mase_profile_read(mase_ctx* ctx, double* total_ms, int64_t* launches, int64_t* units);

/* ---- sizes and structure exports (work on host-only contexts too) ---- */

enum {
  MASE_INFO_N_GAMMA = 0,      /* number of boundary variables (slack angle excluded) */
  MASE_INFO_N_BOUNDARY_BUS,   /* number of boundary buses */
  MASE_INFO_GAMMA_TAIL,       /* buses in the dense block of the boundary system */
  MASE_INFO_NNZ_FACTOR,       /* doubles of packed factor storage per snapshot */
  MASE_INFO_MAX_LEVELS,       /* deepest level schedule over areas */
  MASE_INFO_FLOPS_LOCAL,      /* flops per snapshot-iteration, local elimination */
  MASE_INFO_FLOPS_GAMMA,      /* flops per snapshot-iteration, boundary solve */
  MASE_INFO_BYTES_ASSEMBLY,   /* algorithmic HBM bytes per snapshot of assembly */
  MASE_INFO_N_SNAP,
  MASE_INFO_N_AREA,
  MASE_INFO_BYTES_CONDENSE,   /* algorithmic HBM bytes per snapshot of local elimination */
  MASE_INFO_FLOPS_DENSE,      /* flops per snapshot of the dense boundary block */
  MASE_INFO_BYTES_BACKSOLVE,  /* algorithmic HBM bytes per snapshot of back substitution */
  MASE_INFO_FLOPS_GAMMA_SPARSE, /* flops per snapshot, sparse part of the boundary solve */
  MASE_INFO_GAMMA_LEVELS,     /* elimination levels of the boundary system's sparse part */
  MASE_INFO_GAMMA_SUPERNODES, /* supernodes of the boundary system's sparse part */
  MASE_INFO_GAMMA_SUPERNODAL, /* 1 if the boundary elimination runs supernodal (else the
                                 level schedule) */
  MASE_INFO_PIPELINE_GROUPS,  /* snapshot groups of mase_solve's pipelined schedule */
  MASE_INFO_GAMMA_SUBTREE_GROUPS, /* workgroups per snapshot of the supernodal boundary
                                     elimination: groups of independent elimination subtrees
                                     (the environment variable MASE_SNODE_GROUPS caps it) */
  MASE_INFO_GAMMA_DENSE_PANEL,    /* columns per LDS panel of the boundary system's dense block
                                     (0: panels read from HBM); the autotuner may change it */
  MASE_INFO_AREA_LDS,             /* areas whose elimination holds their packed storage in LDS (the
                                     others run the level engine over HBM); 0 unless the
                                     environment variable MASE_AREA_LDS=1 was set at creation */
  MASE_INFO_ELIM_THREADS          /* threads per workgroup of the LDS elimination and back
                                     substitution (0: per launch class, 1024 for areas that take a
                                     whole CU's LDS, 512 up to four per CU, else 256); the
                                     autotuner may set 256, 512 or 1024 for all */
};
int mase_info(const mase_ctx* ctx, int32_t what, int64_t* value);

enum {
  MASE_MAP_BOUNDARY_FLAG = 0, /* [n_bus]: 1 if the bus is a boundary bus (area ignored) */
  MASE_MAP_MEAS_AREA = 1,     /* [n_meas]: owning area of each measurement (area ignored) */
  MASE_MAP_GAMMA_VARS = 2,    /* [n_gamma]: global variable ids of Gamma (area ignored) */
  MASE_MAP_LOCAL_VARS = 3,    /* area's local variable ids, canonical order */
  MASE_MAP_N_INTERNAL = 4,    /* [1]: number of internal variables of the area */
  MASE_MAP_E = 5              /* area's E_k: Gamma index of each local boundary variable */
};
/*
 * Copy one map into buf (capacity cap entries); *len receives the full
 * length.  Fails with MASE_ERR_ARG if cap is too small (then *len is set).
 */
int mase_export_map(const mase_ctx* ctx, int32_t kind, int32_t area, int32_t* buf,
                    int64_t cap, int64_t* len);

/*
 * Symbolic pattern of G^k (Eq. 7) over the area's local variables in
 * canonical order, as CSR with sorted columns: rowptr [n_local + 1],
 * colidx [cap].  *nnz receives the entry count.
 */
int mase_export_pattern(const mase_ctx* ctx, int32_t area, int32_t* rowptr,
                        int32_t* colidx, int64_t cap, int64_t* nnz);

/* ---- stage-level entry points (together they make one mase_gn_iter) ---- */

/* Stage 1: assemble G^k, b^k for every area and active snapshot (Eq. 7). */
int mase_stage_assemble(mase_ctx* ctx);
/* Stage 2: eliminate internals, leaving S_b^k and bhat_b^k (Eq. 8-10). */
int mase_stage_condense(mase_ctx* ctx);
/* Stage 3a: assemble S_Gamma and bhat_Gamma from the areas (Eq. 11). */
int mase_stage_gamma_assemble(mase_ctx* ctx);
/* Stage 3b: factor S_Gamma in place and solve for dx_Gamma. */
int mase_stage_gamma_solve(mase_ctx* ctx);
/* Stage 4: scatter-back, interior recovery (Eq. 8), x += dx, convergence;
 * max_abs_dx [n_snap] (host, may be NULL) as in mase_gn_iter. */
int mase_stage_update(mase_ctx* ctx, double* max_abs_dx);

/*
 * Debug reads of stage results for one snapshot (host buffers, canonical
 * orders, dense row-major, both triangles filled):
 *   mase_read_local_system  after stage 1: G^k [n_local x n_local], b^k [n_local]
 *   mase_read_schur         after stage 2: S_b^k [n_b x n_b], bhat_b^k [n_b]
 *   mase_read_gamma_system  after stage 3a: S_Gamma [n_gamma x n_gamma], bhat_Gamma
 *   mase_read_step          after stage 4: dx [2 n_bus] by global variable id
 *                           (entry 2*slack is 0)
 * The values are overwritten by later stages (factorisations work in place).
 */
int mase_read_local_system(mase_ctx* ctx, int32_t snap, int32_t area, double* G, double* b);
int mase_read_schur(mase_ctx* ctx, int32_t snap, int32_t area, double* S, double* bhat);
int mase_read_gamma_system(mase_ctx* ctx, int32_t snap, double* S, double* bhat);
int mase_read_step(mase_ctx* ctx, int32_t snap, double* dx);

#ifdef __cplusplus
}
#endif
#endif /* MASE_H */
