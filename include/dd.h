/*
 * dd.h -- C ABI of the MI355X Lagrange-decomposition dual solver for binary programs.
 *
 * The library implements the data-parallel hot path of generalized min-marginal
 * averaging (Alg. 1 of "DOGE-Train", with its BlockUpdate backpropagation, Alg. 2):
 * every constraint row becomes a binary decision diagram (App. B), one dual
 * iteration is a forward and a backward pass of min-sum sweeps over all of them,
 * and the dual lower bound (D) is reduced on the device.
 *
 * Conventions shared by every entry point
 *  - Status: every function returns 0 (DD_OK) or a negative DD_E_* code; nothing
 *    throws across the ABI.  dd_last_error() returns a thread-local message about
 *    the last failure on the calling thread.
 *  - Edges: a Lagrange multiplier lambda_ij (variable i, row j) is an edge.  Arrays
 *    indexed by edge use the canonical order: rows in input order, the variables of
 *    each row in ascending index order.  Rows given with unsorted columns are sorted
 *    (coefficients follow); duplicate columns are rejected.
 *  - Memory: pointers documented "device" must point to device memory of the
 *    instance's GPU, allocated and owned by the caller, of the stated length; the
 *    library reads or writes them in stream order on the given stream and keeps no
 *    reference after the call.  "host" pointers are read or written before the call
 *    returns.  All inputs are copied; the instance owns its device buffers and frees
 *    them in dd_destroy.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Functions that return a host scalar synchronize that stream.
 *  - Numbers: all device-side arithmetic is IEEE fp32; reported bounds are fp64 sums
 *    of fp32 terms.
 *  - Readings of the paper (stated once here, used throughout):
 *      * a forward pass visits the variables of each row in ascending index order
 *        and a backward pass in descending order (blocks B_1..B_u = hop positions);
 *      * the deferred term alpha_ij * sum_{k in J_i} M_ik of Alg. 1 uses the M of
 *        the previous pass for the whole pass (pass-start snapshot), as the
 *        feasibility half of the proof of Prop. 1 requires;
 *      * lambda starts at c_i / |J_i| and M at 0;
 *      * the lower bound is (D) at the flushed multipliers
 *        lambda_bar_ij = lambda_ij + alpha_ij * sum_k M_ik, plus min(0, c_i) for every
 *        variable that appears in no row.
 */
#ifndef DD_H
#define DD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DD_OK = 0,
    DD_E_ARG = -1,         /* bad argument: null pointer, index out of range, duplicate column, bad sense */
    DD_E_INFEASIBLE = -2,  /* a row has no feasible assignment */
    DD_E_FORCED = -3,      /* a row fixes one of its variables (a min-marginal would be infinite) */
    DD_E_PARAM = -4,       /* non-finite cost, omega outside [0,1], non-finite or negative alpha */
    DD_E_HIP = -5,         /* a HIP runtime call failed (message has the HIP error string) */
    DD_E_UNSUPPORTED = -6, /* a row's decision diagram is wider than the kernels support */
    DD_E_OOM = -7,         /* device or host allocation failed */
    DD_E_NONFINITE = -8,   /* a reduced bound is not finite */
    DD_E_STATE = -9,       /* call out of order (e.g. backward without a recorded forward) */
    DD_E_CHECKPOINT = -10  /* a checkpoint of the unrolled forward changed, or recomputing from it did not
                              reproduce the next one (dd_backward) */
};

/* Binary program (Def. 1): min <c, x> s.t. each row  sum_p coef[p] x[col[p]]  (sense)  rhs,
 * x in {0,1}^n; sense -1 means <=, 0 means ==, +1 means >=.  Rows in CSR form: row j
 * holds entries row_ptr[j] .. row_ptr[j+1]-1.  All host pointers. */
typedef struct {
    int32_t n;              /* number of variables */
    const double *c;        /* [n] costs */
    int32_t m;              /* number of rows (subproblems) */
    const int64_t *row_ptr; /* [m+1], row_ptr[0] = 0, non-decreasing */
    const int32_t *col;     /* [nnz] variable ids in [0, n) */
    const int32_t *coef;    /* [nnz] non-zero integer coefficients */
    const int8_t *sense;    /* [m] */
    const int64_t *rhs;     /* [m] */
} dd_problem;

/* Launch options; zero means "default".  Pass NULL for all defaults. */
typedef struct {
    int32_t nodes_per_lane; /* target decision-diagram nodes per lane per hop (team size choice), default 4 */
    int32_t waves_per_block;/* max waves (tiles) per workgroup, 1..4, default 4 (DD_E_ARG otherwise) */
    int32_t ckpt_every;     /* iterations between adjoint checkpoints, default 5 */
    int32_t lds_budget;     /* max LDS bytes per workgroup, default 64 KiB */
    int32_t no_graphs;      /* nonzero: dd_run, the unrolled forward and the backward sweep launch every
                               kernel themselves instead of replaying captured graphs */
    int32_t adj_route_dense;/* nonzero: the reverse sweeps of one-wave diagrams route every level node by
                               node instead of through their per-level lists of nonzero adjoints (the
                               path taken by levels whose lists overflow); for checking that path */
    int32_t adj_replay;     /* nonzero: the checkpointed backward sweep recomputes each segment's pass
                               inputs and replays every pass for its adjoint instead of storing the
                               segment's node costs (no device memory beyond the checkpoints) */
    int32_t lb_every;       /* default iterations between the bounds dd_run_trace records, default 1 */
    int64_t max_device_bytes; /* cap on the device memory the instance may hold, 0 = none: an allocation
                                 that would pass it fails with DD_E_OOM (at create, or later when reverse
                                 mode, a stored trajectory or a feature first needs memory) */
} dd_options;
/* Tile and launch shapes have no option of their own: one wavefront processes one tile of 64 / P
 * diagrams (P, the lanes per diagram, follows from nodes_per_lane), waves_per_block sets the
 * workgroup size, passes are hop-synchronous inside a wave (no hop blocking), and every result is
 * deterministic (fixed reduction orders, no floating-point atomics in device memory), so there is no
 * non-deterministic mode to choose. */

typedef struct {
    int64_t n, m, edges;    /* variables, rows, edges (Lagrange multipliers) */
    int64_t nodes;          /* decision-diagram nodes (non-terminal) */
    int64_t arcs;           /* 2 * nodes, arcs to the 0-terminal included */
    int64_t node_slots;     /* nodes plus layout padding, as stored on the device */
    int64_t edge_slots;     /* edges plus layout padding */
    int64_t tiles;          /* wavefront tiles */
    int32_t max_width;      /* widest level of any diagram */
    int32_t max_len;        /* longest row */
    int32_t classes;        /* kernel specialisations used */
    int32_t uncovered;      /* variables in no row */
    int64_t device_bytes;   /* bytes the instance holds on the device */
    int64_t coded_levels;   /* levels of one-wave diagrams whose passes read the topology in one byte
                               per node (child-code steps; see DevTables::tcode) */
    int64_t raw_levels;     /* levels of one-wave diagrams read in four bytes per node (steps that do
                               not fit a nibble) */
} dd_stats;

typedef struct dd_instance dd_instance;

/* Thread-local message describing the last error on this thread ("" if none). */
const char *dd_last_error(void);

/* Compile every row to a quasi-reduced ordered decision diagram (App. B: every
 * root-to-1 path visits one node per variable; paths are exactly X_j), lay them out
 * for the device, upload, and reset the solver (lambda = c/|J_i|, M = 0, omega = 0.5,
 * alpha = 1/|J_i|: the special case of the Remark after Alg. 1's description).
 * Uses the current HIP device.  Errors: DD_E_ARG, DD_E_PARAM, DD_E_INFEASIBLE,
 * DD_E_FORCED, DD_E_UNSUPPORTED, DD_E_OOM, DD_E_HIP.  On error *out is NULL. */
int dd_create(const dd_problem *prob, const dd_options *opt, void *stream, dd_instance **out);

/* Free all device and host memory of the instance (NULL is accepted). */
int dd_destroy(dd_instance *h);

/* Sizes of the instance (host struct). */
int dd_get_stats(const dd_instance *h, dd_stats *out);

/* Number of edges (Lagrange multipliers lambda_ij, one per variable i of row j: the coupling of the
 * decomposition, Sec. "Lagrange decomposition").  Host. */
int dd_num_edges(const dd_instance *h, int64_t *E);

/* Canonical edge e -> (variable, row): the pairs (i, j), i in I_j, that index the Lagrange
 * multipliers (Sec. "Lagrange decomposition"); host arrays of length edges. */
int dd_edge_map(const dd_instance *h, int32_t *var_out, int32_t *row_out);

/* Set the damping factors omega_ij (in [0,1], Prop. 1) and averaging weights alpha_ij
 * (>= 0; Prop. 1 also needs sum_{j in J_i} alpha_ij = 1, which the caller ensures,
 * e.g. through dd_seg_softmax).  Device arrays [edges], canonical order, copied. */
int dd_set_params(dd_instance *h, const float *omega, const float *alpha, void *stream);

/* alpha_{i.} = softmax over J_i of alpha_hat_{i.} (the transform of Alg. 3 that makes
 * alpha a convex combination).  Device arrays [edges], canonical order. */
int dd_seg_softmax(dd_instance *h, const float *alpha_hat, float *alpha_out, void *stream);

/* Back to the start state of Alg. 1: lambda = c_i/|J_i| (a feasible start; the paper leaves the
 * initialization to the caller), M = 0 (Alg. 1, initialization), shortest-path costs recomputed. */
int dd_reset(dd_instance *h, void *stream);

/* Replace the solver state (lambda, M) of Alg. 1 (device arrays [edges], canonical order): a test hook
 * and the resume point of a round that starts elsewhere (Sec. "Overall pipeline"); shortest-path
 * costs are recomputed.  Feasibility (Prop. 1) is the caller's: sum_j (lambda_ij + M_ij) = c_i. */
int dd_set_state(dd_instance *h, const float *lambda, const float *M, void *stream);

/* Read the state (lambda, M) that Alg. 1 returns into device arrays [edges] (canonical order).
 * flushed != 0 returns lambda_bar = lambda + alpha * S instead of lambda: the deferred term applied,
 * the dual-feasible multipliers at which the bound (D) is evaluated.  M_out may be NULL. */
int dd_get_state(dd_instance *h, float *lambda_out, float *M_out, int32_t flushed, void *stream);

/* T iterations of Alg. 1: each a forward pass (hops in ascending variable order)
 * then a backward pass; every pass applies BlockUpdate to all hops of all rows.
 * For T >= 2 the iterations are replayed from HIP graphs captured on first use (one
 * of 1 iteration, one of 8), unless the instance was created with no_graphs or is
 * profiling; the launches, and so the results, are the same either way. */
int dd_run(dd_instance *h, int32_t T, void *stream);

/* One pass of Alg. 1: direction 0 = forward, 1 = backward.  A pass reads the other side's
 * shortest-path costs at its input multipliers (eq. 8 for the hops it has not visited yet): B for a
 * forward pass, F for a backward pass.  A pass of the other direction leaves them in place; when the
 * previous call did not (two passes of one direction in a row, or a call that moved the multipliers
 * or reused the node arrays: dd_set_state, dd_reset, dd_min_marginals, dd_pass_vjp, dd_backward, ...)
 * they are recomputed first, with one more sweep. */
int dd_run_pass(dd_instance *h, int32_t direction, void *stream);

/* Lower bound (D) at lambda_bar plus the uncovered-variable constant (into *lb), and
 * the lifted-representation bound of Prop. 1's proof,
 * D_L = sum_j E^j(lambda) + sum_e min(0, M_e) + the same constant (into *dl, may be NULL).
 * Synchronizes the stream.  DD_E_NONFINITE if a bound is not finite. */
int dd_lower_bound(dd_instance *h, double *lb, double *dl, void *stream);

/* T iterations of Alg. 1 (as dd_run) recording the lower bound (as dd_lower_bound, the constant of
 * variables in no row included) after every lb_every iterations (0: the instance's lb_every option):
 * lb_dev[i] (device, fp64, caller-allocated, floor(T / lb_every) entries) is the bound after
 * (i + 1) lb_every iterations.  Asynchronous: nothing is copied to the host and the stream is not
 * synchronized, so a caller reads the whole trajectory once at the end. */
int dd_run_trace(dd_instance *h, int32_t T, int32_t lb_every, double *lb_dev, void *stream);

/* Per-row energies E^j(lambda_bar) (eq. 1) into a device array [m]. */
int dd_row_energies(dd_instance *h, float *E_out, void *stream);

/* Min-marginals m^0, m^1 of every edge at lambda_bar (eq. 8), device arrays [edges]. */
int dd_min_marginals(dd_instance *h, float *m0_out, float *m1_out, void *stream);

/* Replace the costs c (device array [n], f32) and reset the solver (lambda = c/|J_i|, M = 0). */
int dd_set_costs(dd_instance *h, const float *c, void *stream);

/* ---- Reverse mode (Alg. 2, Prop. 2; loss = the dual objective, Sec. "Loss") ---------------- */

/* Reset, then run T iterations of Alg. 1 keeping the state (lambda, M) every ckpt_every
 * iterations (0: the instance default), and return the lower bound of the final state.
 * ckpt_every = -1 keeps the whole trajectory on the device instead: the node costs F or B that
 * every pass wrote (2T + 1 arrays of the diagrams' node count, f32) and the state before every
 * pass, so dd_backward recomputes no pass (DD_E_OOM, with nothing run, when the free device
 * memory is short; the arrays stay allocated with the instance for later calls).
 * Records what dd_backward needs; any later call that changes the state (a pass, reset,
 * set_state, set_params, set_costs) invalidates the record.  With checkpoints, the deferred sums
 * S of every pass are kept too (2T arrays of n floats) for the recomputed segments, and when the
 * 2K + 1 node-cost arrays that dd_backward recomputes a segment into fit on the device, the last
 * segment runs with the recording passes straight into them (same bits), so that dd_backward
 * does not recompute it; the final B is then copied back to the instance.  The launches
 * after the reset are captured into a HIP graph the first time (T, ckpt_every) is seen with the
 * same buffers and replayed afterwards (not while profiling or with no_graphs); results are the
 * same bits either way. */
int dd_forward_unrolled(dd_instance *h, int32_t T, int32_t ckpt_every, double *lb, void *stream);

/* Gradient of dlb * LB(after the recorded T iterations) with respect to omega, alpha and c:
 * the seed dLB/dlambda_bar is the argmin assignment of every row (Sec. "Loss"), the flush
 * lambda_bar = lambda + alpha*S is differentiated, then every pass in reverse with Alg. 2
 * (each segment between checkpoints is recomputed, keeping its node costs, its states and its
 * passes' argmins on the device when 2K + 1 node-cost arrays fit -- they stay allocated with the
 * instance -- or else, and always with the adj_replay option, replaying every pass bit for bit
 * to recover them; the results are the same bits), and finally lambda_0 = c/|J_i|; a variable
 * in no row contributes
 * dlb * [c_i < 0].  Subgradients at ties: lo arcs before hi arcs, lower node indices first.
 * Outputs are device arrays (may be NULL): d_omega, d_alpha [edges] canonical, d_c [n].
 * Leaves the solver at the final state.  DD_E_STATE without a valid record.  The launches up to
 * the start-state adjoints replay a captured graph as dd_forward_unrolled's do (dlb is read from
 * device memory, so one graph serves every seed); the call ends with a host wait for the
 * checkpoint verification flag. */
int dd_backward(dd_instance *h, double dlb, float *d_omega, float *d_alpha, float *d_c, void *stream);

/* Test hook for the checkpoint verification: adds 1 to the first multiplier slot of checkpoint
 * `index` (0 .. ceil(T / K)) of the recorded checkpointed forward, so that the next dd_backward that
 * reads it returns DD_E_CHECKPOINT (every checkpoint is verified when it is read; the start of a
 * last segment that the forward kept is read only by a second dd_backward of the same record).
 * DD_E_STATE without such a record.  Synchronizes the device. */
int dd_corrupt_checkpoint(dd_instance *h, int32_t index);

/* Serial number of the recorded unrolled forward, for callers that hold several records of one
 * instance (each autograd node of a graph): every successful dd_forward_unrolled* takes the next
 * serial; *serial = -1 when no record is valid (none made, or the state changed since).  A caller
 * that kept the serial of its forward and finds another one here knows that dd_backward would
 * differentiate a later forward, not its own.  Host only. */
int dd_record_serial(const dd_instance *h, int64_t *serial);

/* Alg. 2 applied to one whole pass (direction 0 forward, 1 backward): given the pass input
 * (lam_in, M_in) and the adjoints of its outputs (dlam_out, dM_out), write the adjoints of the
 * inputs (dlam_in, dM_in) and of alpha and omega (d_alpha, d_omega, not accumulated).  All
 * device arrays [edges], canonical order.  The state is left at the pass output. */
int dd_pass_vjp(dd_instance *h, int32_t direction, const float *lam_in, const float *M_in, const float *dlam_out,
                const float *dM_out, float *dlam_in, float *dM_in, float *d_alpha, float *d_omega, void *stream);

/* As dd_forward_unrolled, but the T iterations start from the instance's current state (lambda, M)
 * instead of the reset state: one round of the paper's pipeline (Sec. "Overall pipeline") starts
 * where the previous round stopped, after the non-parametric update. */
int dd_forward_unrolled_from_state(dd_instance *h, int32_t T, int32_t ckpt_every, double *lb, void *stream);

/* As dd_backward, but also returning the adjoints of the state the recorded forward started from:
 * d_lam0, d_M0 (device arrays [edges], canonical order; any output may be NULL).  After a forward
 * from the reset state d_lam0 is the adjoint of lambda_0 = c/|J_i|; dd_backward's d_c needs such a
 * forward (DD_E_ARG after dd_forward_unrolled_from_state). */
int dd_backward_state(dd_instance *h, double dlb, float *d_omega, float *d_alpha, float *d_lam0, float *d_M0,
                      void *stream);

/* Output transforms of the parameter predictor (Alg. 3, last lines): omega = sigmoid(omega_hat),
 * alpha = softmax over J_i of alpha_hat (as dd_seg_softmax), theta = theta_hat minus its mean over
 * J_i (dual feasibility).  Device arrays [edges], canonical order; theta_hat and theta may both be
 * NULL. */
int dd_param_transform(dd_instance *h, const float *omega_hat, const float *alpha_hat, const float *theta_hat,
                       float *omega, float *alpha, float *theta, void *stream);

/* Adjoint of dd_param_transform: given its outputs omega, alpha and the adjoints d_omega, d_alpha,
 * d_theta, writes d_omega_hat = d_omega * omega (1 - omega), d_alpha_hat (softmax VJP) and
 * d_theta_hat = d_theta minus its mean over J_i (the centring is symmetric and idempotent).
 * d_theta and d_theta_hat may both be NULL. */
int dd_param_transform_vjp(dd_instance *h, const float *omega, const float *alpha, const float *d_omega,
                           const float *d_alpha, const float *d_theta, float *d_omega_hat, float *d_alpha_hat,
                           float *d_theta_hat, void *stream);

/* Non-parametric update (eq. 2): lambda_ij += theta_hat_ij - (1/|J_i|) sum_{k in J_i} theta_hat_ik on
 * the current state (M unchanged; sum_j (lambda_ij + M_ij) is preserved).  theta_hat: device array
 * [edges], canonical order.  Its adjoint is the same centring of d_lambda (dd_param_transform_vjp's
 * theta part). */
int dd_nonparam_update(dd_instance *h, const float *theta_hat, void *stream);

/* d_alpha_hat = VJP of alpha = softmax over J_i (dd_seg_softmax): alpha_e (d_alpha_e - sum_k alpha_k d_alpha_k).
 * Device arrays [edges], canonical order. */
int dd_seg_softmax_vjp(dd_instance *h, const float *alpha, const float *d_alpha, float *d_alpha_hat, void *stream);

/* ---- Solver features (the appendix's feature table) ----------------------------------------- */

/* Smoothed subproblems at temperature tau > 0 (the smoothing of the feature table, read as a
 * soft-min): E_tau^j = -tau log sum_{x in X_j} exp(-<lambda_.j, x>/tau) into E_out [m] (may be NULL),
 * and its gradient, the Gibbs marginals P(x_i = 1) on X_j, into p_out [edges] (canonical order),
 * at lambda (flushed = 0) or at lambda_bar (flushed != 0).  Device arrays.  The first call
 * allocates a node-sized scratch array kept until dd_destroy. */
int dd_smoothed(dd_instance *h, float tau, int32_t flushed, float *E_out, float *p_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): dd_smoothed, with the node scratch of its sweeps taken
 * from a 16 MiB array per GPU that the library reserves when it is loaded and holds until the
 * process ends, instead of an array allocated on first use.  Allocates nothing; same kernels and
 * results as dd_smoothed.  Limit: instances of at most 4,194,240 node slots (dd_stats.node_slots);
 * larger ones get DD_E_ARG.  The current device must be the instance's (DD_E_ARG otherwise).  Every
 * call on one GPU uses that GPU's one array: calls that overlap on a GPU (other streams or threads)
 * race on it and must be serialized by the caller. */
int dd_smoothed_noalloc(dd_instance *h, float tau, int32_t flushed, float *E_out, float *p_out, void *stream);

/* Minimizing assignment of every row (a subgradient of the dual objective, Sec. "Loss"), 0/1 per
 * edge into x_out [edges] (f32, canonical order), at lambda or lambda_bar; ties: lo arcs first. */
int dd_argmin_assignment(dd_instance *h, int32_t flushed, float *x_out, void *stream);

/* ---- Test-time driver (Sec. "Overall pipeline", Sec. "Evaluation") -------------------------- */

/* Rounds of T iterations of Alg. 1 (as dd_run) with the lower bound after each: stops after
 * max_rounds rounds or after the first round whose bound improves on the previous one by less than
 * rel_tol times its magnitude (the paper switches networks at a relative improvement of 1e-6).
 * lb_trace, ms_trace: host arrays [max_rounds + 1] receiving the bound before the first round and
 * after each round, with the milliseconds elapsed since the call began (host clock, taken after the
 * bound's synchronization); *rounds receives the number of rounds run. */
int dd_solve(dd_instance *h, int32_t T, int32_t max_rounds, double rel_tol, double *lb_trace, double *ms_trace,
             int32_t *rounds, void *stream);

/* Relative dual gap of a trace (Sec. "Evaluation"): g_i = min((d_star - lb_i) / (d_star - lb_0), 1)
 * into g_out [k] (may be NULL; 0 when d_star <= lb_0), and its integral over time in seconds with each
 * value held until the next, g_I = sum_i g_i (ms_{i+1} - ms_i) / 1000.  Host-only. */
int dd_gap_integral(const double *lb, const double *ms, int32_t k, double d_star, double *g_out, double *g_integral);

/* Nodes of each row's diagram, host array [m] (0 for an empty row). */
int dd_row_nodes(const dd_instance *h, int64_t *nodes_out);

/* Per-kernel timing of the instance's own launches, for roofline reporting.
 * dd_profile_begin starts recording a HIP event pair around every kernel launch the
 * instance makes (pool of `max_launches` pairs, created here so recording allocates
 * nothing); dd_profile_end synchronizes the device, stops recording and aggregates
 * by kernel: out[k] gets the kernel's name (as the profiler shows it), launch count,
 * summed duration and the algorithmic bytes one launch must move (the per-node and
 * per-edge traffic of the method times the nodes and edges the launch covers).
 * *count receives the number of kernels (at most cap are written). */
typedef struct {
    char name[96];
    int64_t launches;
    double total_ms;
    double bytes_per_launch;
} dd_kernel_time;
int dd_profile_begin(dd_instance *h, int32_t max_launches);
int dd_profile_end(dd_instance *h, dd_kernel_time *out, int32_t cap, int32_t *count);

/* ---- Launch shapes -------------------------------------------------------------------------- */

/* Kernel specialisation classes of the instance and their launch shapes.  Class c's entry is
 * out[6c .. 6c+5] = {team size P, register rows RMAX, waves per workgroup of the forward and
 * backward pass kernels, workgroups of the forward and backward pass kernels (0: one wave
 * per tile; otherwise that many resident workgroups whose waves walk the tile list)}.
 * *count receives the number of classes; at most cap entries are written. */
int dd_get_launch(const dd_instance *h, int32_t *out, int32_t cap, int32_t *count);

/* Set class c's pass-kernel launch shape (waves per workgroup 1..4 within the LDS budget;
 * grid 0 or a positive workgroup count).  The arithmetic, and so every result, does not
 * depend on the shape.  DD_E_ARG on an out-of-range class or an infeasible shape. */
int dd_set_launch(dd_instance *h, int32_t c, int32_t wpb_f, int32_t wpb_b, int32_t grid_f, int32_t grid_b);

/* Autotuner: time the forward and backward update kernels of every class over a small set
 * of launch shapes (waves per workgroup 1, 2, 4 x {one wave per tile, a resident grid of the size the
 * CUs hold at once}) and keep the fastest.  cache_path (may be NULL) names a text file: a
 * line "signature<TAB>shapes" per tuned instance shape, signature = device architecture and
 * every class's (P, RMAX, tiles, nodes); a hit is applied without timing (*from_cache = 1).
 * New results are appended.  The solver state is restored afterwards. */
int dd_autotune(dd_instance *h, const char *cache_path, int32_t *from_cache, void *stream);

/* ---- Batches: many programs packed into one instance ---------------------------------------- */

/* A batch is the disjoint union of k programs (variables and rows of program q follow those
 * of q-1): the mini-batches of the training loop (Sec. "Loss": the loss is averaged over a
 * mini-batch of instances; Table 5 gives the batch sizes).  Every pass over the batch is one launch
 * per kernel class over all programs, and rows of different programs share tiles.  Since the
 * programs share no variable, each one's iterates are those it would have alone (Alg. 1 couples
 * rows only through shared variables).  dd_batch_instance returns the packed instance (owned by the
 * batch) for every per-instance call; its edge, variable and row arrays are the programs' canonical
 * arrays concatenated in batch order.  The batch is built from the programs (rows are compiled into
 * shared tiles), not from existing instances, which keep no copy of their rows. */
typedef struct dd_batch dd_batch;
int dd_batch_create(const dd_problem *probs, int32_t k, const dd_options *opt, void *stream, dd_batch **out);
int dd_batch_destroy(dd_batch *b);
dd_instance *dd_batch_instance(dd_batch *b);
/* Offsets of program q's variables, rows and edges: host arrays [k+1] each (may be NULL). */
int dd_batch_offsets(const dd_batch *b, int64_t *var_off, int64_t *row_off, int64_t *edge_off);
/* T iterations of Alg. 1 over every program (graph replays as in dd_run). */
int dd_batch_run(dd_batch *b, int32_t T, void *stream);
/* Per-program lower bounds (D) (as dd_lower_bound, each with its own uncovered-variable
 * constant): lbs[k] and, if not NULL, dls[k] (D_L).  Host arrays; synchronizes the stream. */
int dd_batch_lower_bounds(dd_batch *b, double *lbs, double *dls, void *stream);

/* Host-only helper: compile row `row` of prob and return its diagram.  width[L] gets
 * the node count per level (L = row length); arcs[nodes] gets, level by level, each
 * node's (lo | hi << 16) child codes, where a code c < width[l+1] is a node of the
 * next level, c == width[l+1] the 0-terminal and c == width[l+1] + 1 the 1-terminal
 * (width[L] taken as 0).  *nodes receives the node count; arcs may be NULL to query
 * it.  cap is the capacity of arcs.  No GPU needed. */
int dd_compile_row(const dd_problem *prob, int32_t row, int32_t *width, uint32_t *arcs, int64_t cap,
                   int64_t *nodes);

#ifdef __cplusplus
}
#endif
#endif /* DD_H */
