/*
 * mwu.h -- C ABI of the MI355X (gfx950) multiplicative-weight-update solver
 * for positive linear programs.
 *
 * Method: Ju, Yesil, Sun, Chekuri, Solomonik, "Efficient Parallel
 * Implementation of the Multiplicative Weight Update Method for Graph-based
 * Linear Programs" (arXiv 2307.03307):
 *   - problem forms: general LP (eq. LPDef, Section 1), normalized mixed
 *     packing/covering feasibility (eq. NormFeasibleLP, Section 2.2), pure
 *     packing and pure covering with the objective embedded as one extra row
 *     and M searched (end of Section 2.2);
 *   - graph LPs: matching / bipartite matching, dominating set, vertex cover,
 *     densest subgraph with D searched (Section 3);
 *   - iteration: Algorithm 2 with the step-size search of Algorithm 3
 *     (Section 4), or the standard step alpha = 1 (Algorithm 1).
 *
 * Conventions shared by every entry point
 *   - Every function returns an mwu_status: 0 (MWU_OK) or a negative error.
 *     Solve outcomes (feasible, infeasible, iteration cap) are not errors;
 *     they are reported in mwu_result_info.status.
 *   - Host pointers are plain host memory unless stated otherwise.  Inputs are
 *     deep-copied by mwu_create*; the caller may free them on return.
 *   - A handle owns all device memory until mwu_destroy.  A handle is not
 *     thread-safe; distinct handles are independent.
 *   - All indices are 0-based.  Device-side indices are 32-bit: every count
 *     (rows, columns, nonzeros, vertices, edges) must be below 2^31 - 1,
 *     otherwise MWU_ERR_TOO_LARGE.
 */
#ifndef MWU_H
#define MWU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mwu_status;

/* error codes (negative) */
#define MWU_OK                 0
#define MWU_ERR_INVALID_ARG   -1  /* NULL where not allowed, eps outside (0,1), size mismatch */
#define MWU_ERR_NEGATIVE_ENTRY -2 /* a matrix value < 0 */
#define MWU_ERR_NONFINITE     -3  /* NaN or infinity in values, b or c */
#define MWU_ERR_BAD_RHS       -4  /* some b_i <= 0 or c_j <= 0 */
#define MWU_ERR_GRAPH         -5  /* self-loop, duplicate edge or vertex id out of range */
#define MWU_ERR_TOO_LARGE     -6  /* a count does not fit the 32-bit device indices */
#define MWU_ERR_OOM           -7  /* device or host allocation failed */
#define MWU_ERR_DEVICE        -8  /* HIP runtime error, or no gfx950 device */
#define MWU_ERR_UNBOUNDED     -9  /* packing column with no nonzero: the LP is unbounded */
#define MWU_ERR_STATE        -10  /* call not valid for this handle (e.g. probe API before a probe) */

/* solve outcome, mwu_result_info.status */
#define MWU_CERTIFIED            0  /* returned x is feasible and within (1+eps) of OPT */
#define MWU_FEASIBLE_UNCERTIFIED 1  /* feasible x, bracket not closed (probe cap or iteration cap) */
#define MWU_INFEASIBLE           2  /* single-probe mode: the feasibility LP is infeasible */
#define MWU_MAX_ITER             3  /* single-probe mode: iteration cap reached */
#define MWU_FEASIBLE_POINT       4  /* single-probe mode (MWU_MIXED with mixed_fixed_lambda): Algorithm 2
                                       stopped with C x >= b_C (Section 4); x_out is that point, not
                                       rescaled, objective_out = max_i (A_P x)_i / b_P,i (its lambda,
                                       at most about (1 + eps) times the lambda asked for), and
                                       max_violation = max{0, max(Px)/lambda - 1, 1 - min(Cx)} of it */

/* probe outcome (mwu_probe_info.status) */
#define MWU_PROBE_RUNNING    0
#define MWU_PROBE_FEASIBLE   1  /* min(Cx) >= 1 reached (Algorithm 2 stop) */
#define MWU_PROBE_INFEASIBLE 2  /* max(d) = 0, or the step search found alpha < 1 */
#define MWU_PROBE_MAX_ITER   3

typedef enum {
    MWU_PACKING = 0,   /* max c^T x  s.t. A x <= b, x >= 0        (eq. LPDef; pure packing, Sec. 2.2) */
    MWU_COVERING = 1,  /* min c^T x  s.t. A x >= b, x >= 0        (pure covering, Sec. 2.2)          */
    MWU_MIXED = 2,     /* min lambda s.t. P x <= lambda b_P, C x >= b_C, x >= 0: the densest
                          subgraph "min D" form (Section 3); with opts.mixed_fixed_lambda > 0 a
                          single feasibility probe P x <= lambda b_P, C x >= b_C (eq. NormFeasibleLP) */
    /* Mixed optimization (last sentence of Section 2.2): max (MIXED_MAX) or
     * min (MIXED_MIN) c^T x s.t. P x <= b_P, C x >= b_C, x >= 0, c > 0
     * required.  The objective is embedded as one more row, (1/M) c^T x >= 1
     * among the covering rows (max) or <= 1 among the packing rows (min), and
     * M is searched: an infeasible probe at M proves OPT < M (max) or
     * OPT > M (min); a feasible one gives x with C x >= b_C and the objective
     * row met, its packing rows (the objective row too when minimizing)
     * within Algorithm 2's (1 + eps).  Results: x_out is the best feasible
     * probe's point, objective_out its c^T x, [lower, upper] the bracket
     * (max: largest feasible M, smallest infeasible M; min: largest
     * infeasible M, smallest feasible M), max_violation its
     * max{0, max_i (P x)_i / b_P,i - 1} (minimizing, the objective row
     * c^T x / M counts among the packing rows).  CERTIFIED when the bracket
     * is within 1 + eps; INFEASIBLE when no probe was feasible (x_out is
     * then all zero).  Maximizing, a column without a packing entry is
     * rejected (MWU_ERR_UNBOUNDED); minimizing, a column without a covering
     * entry is kept and never moves from its start.  Generic CSR engine;
     * probe reuse is not applied. */
    MWU_MIXED_MAX = 3,
    MWU_MIXED_MIN = 4
} mwu_form;

typedef enum {
    MWU_MAT_CSR = 0,          /* explicit CSR: row_ptr (int64, rows+1), col_idx (int32, nnz),
                                 values (double, nnz; NULL = every stored entry is 1)           */
    MWU_MAT_INCIDENCE = 1,    /* M (num_vertices x num_edges) from an edge list: M[u,e] = 1 iff
                                 u is an endpoint of e (eq. incidence, Section 3)                */
    MWU_MAT_INCIDENCE_T = 2,  /* M^T (num_edges x num_vertices): row e reads x_u + x_v (vertex
                                 cover, Section 3)                                               */
    MWU_MAT_EDGE_PAIR = 3,    /* O (num_vertices x 2 num_edges): O[u,2e] = 1 for e = (u,.),
                                 O[v,2e+1] = 1 for e = (.,v) (eq. oddshifted, Section 3)        */
    MWU_MAT_INTERWEAVE = 4    /* W (num_edges x 2 num_edges): W[e,2e] = W[e,2e+1] = 1
                                 (eq. interweaved, Section 3)                                    */
} mwu_matrix_kind;

/* A constraint matrix.  CSR fields are used for MWU_MAT_CSR, edge-list fields
 * for the implicit graph kinds.  Edge lists: vertices 0..num_vertices-1, no
 * self-loops, no duplicate undirected edge (MWU_ERR_GRAPH otherwise); any
 * order and orientation.  Edge e of the caller's list is variable e (and the
 * pair variables 2e, 2e+1) in the caller's order. */
typedef struct {
    mwu_matrix_kind kind;
    int64_t rows, cols;            /* CSR only */
    const int64_t *row_ptr;        /* CSR only */
    const int32_t *col_idx;        /* CSR only */
    const double *values;          /* CSR only, nullable */
    int64_t num_vertices, num_edges;
    const int32_t *edge_u;         /* edge kinds only */
    const int32_t *edge_v;
} mwu_matrix;

/* The LP.  PACKING uses P only, COVERING uses C only, MIXED uses both.
 * b_P (rows of P), b_C (rows of C) and c (columns) are nullable (all ones).
 * Implicit graph kinds are pattern-only 0/1 matrices; passing b or c with
 * them is allowed and materializes the scaled matrix as CSR. */
typedef struct {
    mwu_form form;
    mwu_matrix P, C;
    const double *b_P;
    const double *b_C;
    const double *c;
} mwu_problem;

#define MWU_STEP_STD 0   /* alpha = 1 (Algorithm 1) */
#define MWU_STEP_BIN 1   /* exponential + binary search (Algorithm 3) */
/* Algorithm 3 started at the step the probe accepted last (the setting of
 * the Bin column of Table 2): doubling from there while the test holds, or
 * halving while it fails (never below 1; a failing test at 1 ends the probe
 * as infeasible), then the same bisection.  The first iteration of a probe
 * starts at 1. */
#define MWU_STEP_BIN_WARM 2
/* Newton's method for the step (Section 4.2, the Nwt column of Table 2):
 * Newton steps on g(alpha) = Phi(alpha)/Psi(alpha) - 1 from the step the
 * probe accepted last, g' formed from Psi' and Phi' (averages of P d and C d
 * under the weights of the moved point), each iterate tested once and kept
 * inside the bracket of the values tested so far (2 alpha, hi/2 or
 * sqrt(lo hi) replace an iterate outside it); it stops when the correction
 * is at most eps alpha or after 8 tests, and the values alpha (1-eps)^p are
 * then tested until one passes.  The first iteration of a probe takes
 * Algorithm 3's step; with MWU_FLAG_REUSE a probe after the first starts
 * Newton at the previous probe's last step. */
#define MWU_STEP_NEWTON 3

#define MWU_FP64 0               /* plain: every vector and sum in double */
#define MWU_MIXED_FP32_FP64 1    /* vectors and per-element terms in float; LSE totals, search sums,
                                    step decisions and certificates in double */

#define MWU_FLAG_NO_FACTOR2   1u  /* do not double the step when one side is a single row */
#define MWU_FLAG_GENERIC      2u  /* force the generic CSR engine (no fused graph program) */
#define MWU_FLAG_NO_TUNE      4u  /* batched: take the default layout, time nothing (the default;
                                     overrides MWU_FLAG_TUNE) */
#define MWU_FLAG_TUNE         128u /* batched: choose the layout by a timed sweep (or a known record) */
/* Outer search: every probe after the first starts from the previous probe's
 * iterate, scaled so that its largest packing row (in the new probe's scale)
 * is eps -- the level the Algorithm 1 point starts from -- and, with
 * MWU_STEP_BIN_WARM, searches its first step from the previous probe's last
 * step.  Single-problem handles; the batched program ignores it. */
#define MWU_FLAG_REUSE        8u
/* Drop satisfied covering rows: every iteration leaves out the covering rows
 * with (C x)_i >= 1 (weight 0 in the smoothed minimum, h, Phi and the step
 * search), the line C <- {c_i : c_i^T x < 1} of Algorithms 1 and 2 (Section
 * 2.2, Section 4), which the paper's own experiments leave out.  eta stays
 * that of the full row count.  Single-problem handles; the batched program
 * (no explicit covering rows) ignores it. */
#define MWU_FLAG_DROP_SATISFIED 16u
/* Generic CSR engine: its internal order of the variables and of the rows
 * (no effect on any result's order, which stays the caller's).  By default
 * the engine sorts the columns by their number of nonzeros and the rows of
 * each side by theirs, both descending, when the column lengths are heavy-
 * tailed (at least 4096 columns, the longest at least 32 times the mean):
 * the random gathers of the two products then fall mostly on a compact
 * prefix of hub entries.  KEEP_ORDER never reorders (inputs already laid
 * out for locality, such as banded matrices); LOCALITY_ORDER always does. */
#define MWU_FLAG_KEEP_ORDER     32u
#define MWU_FLAG_LOCALITY_ORDER 64u

typedef struct {
    double eps;                 /* accuracy, default 0.1 (Section 6.2) */
    int32_t max_iter;           /* iterations per probe, default 5000 (Section 6.2) */
    int32_t max_probes;         /* outer search cap, default 64 */
    int32_t step_rule;          /* MWU_STEP_BIN (default), MWU_STEP_BIN_WARM, MWU_STEP_NEWTON or
                                   MWU_STEP_STD */
    int32_t precision;          /* MWU_MIXED_FP32_FP64 (default) or MWU_FP64 */
    int32_t iters_per_launch;   /* iterations captured per graph launch; 0 = default (16 for one
                                   instance, 8 for a batch) */
    int32_t device;             /* HIP device ordinal, default 0 */
    void *hip_stream;           /* hipStream_t to run on; NULL = a stream owned by the handle */
    double mixed_fixed_lambda;  /* MWU_MIXED: > 0 runs one feasibility probe at this lambda */
    uint64_t flags;
    const char *tune_cache;     /* batched: text file of tuned layouts, read and appended;
                                   NULL = layouts are remembered for the process only */
} mwu_options;

typedef struct {
    int32_t status;             /* MWU_CERTIFIED ... MWU_MAX_ITER */
    double objective;           /* c^T x of the returned x (MIXED: lambda of the returned x) */
    double lower_bound;         /* final bracket on OPT */
    double upper_bound;
    int64_t total_iterations;   /* MWU iterations over all probes */
    int64_t final_probe_iterations;
    int64_t search_passes;      /* K-candidate step-search passes over the rows */
    int64_t probes;
    double max_violation;       /* max{0, max(Px)-1, 1-min(Cx)} of the last probe's x (Sec. 6.3) */
    double seconds_solve;       /* wall time of mwu_solve */
    int64_t evaluations;        /* tests Phi(alpha) >= Psi(alpha) the step searches made, counted
                                   as a one-at-a-time Algorithm 3 (Section 4.2) makes them */
} mwu_result_info;

/* Fill *opt with the defaults listed above. */
void mwu_default_options(mwu_options *opt);

/* Validate, normalize (P_ij = A_ij / (b_i c_j), Section 2.1), drop empty rows
 * and (covering) empty columns, canonicalize edge lists, upload to the device
 * and build the transpose plans.  opt is nullable (defaults).  On success
 * *out receives a handle; on error *out is set to NULL. */
mwu_status mwu_create(const mwu_problem *prob, const mwu_options *opt, void **out);

/* Many independent problems solved together (every problem must be a
 * MWU_PACKING problem with P of kind MWU_MAT_INCIDENCE, e.g. bipartite
 * matchings).  Variables and results are concatenated in problem order. */
mwu_status mwu_create_batch(const mwu_problem *probs, int32_t count, const mwu_options *opt,
                            void **out);

/* ---------------------------------------------------------------------------
 * Layout of a batched handle and its autotuner.  The batched passes visit
 * edge tiles (start, column and statistics passes), element tiles of vertex
 * rows (row and search passes) and nnz-balanced vertex tiles (forward
 * product, fixed at BLOCK x 8 nonzeros) with persistent grids.  By default
 * mwu_create_batch takes the built-in layout and times nothing.  With
 * MWU_FLAG_TUNE it takes a layout for the same device, precision and batch
 * shape listed in opt->tune_cache or already known to the process, else one
 * chosen by timed sweeps over the batch itself (one coordinate-descent pass
 * over the four fields below; each candidate runs the whole batched solve
 * from its start for 0.4 s, host polling and probe turnovers included, and is
 * rated by the edge-iterations completed per second; about 8 such windows at
 * create).  On the 512-instance workload the tuned and the built-in layouts
 * solve within a few percent of each other, so the sweep is opt-in.
 * ------------------------------------------------------------------------- */

#define MWU_LAYOUT_DEFAULT 0   /* built-in layout, nothing timed */
#define MWU_LAYOUT_TUNED   1   /* chosen by a sweep at create */
#define MWU_LAYOUT_CACHED  2   /* a sweep's result, found in memory or in the cache file */
#define MWU_LAYOUT_SET     3   /* set by mwu_batch_set_layout */

typedef struct {
    int32_t tile_edges;          /* edges per edge tile: multiple of 256 in [256, 65536] */
    int32_t tile_vertices;       /* vertices per element tile: multiple of 256 in [256, 65536] */
    int32_t workgroups_per_cu;   /* cap on resident persistent workgroups per CU: 1..16 */
    int32_t search_launches;     /* step-search passes launched per iteration slot: 1..4 */
    int32_t source;              /* MWU_LAYOUT_* (output only) */
    int32_t candidates_timed;    /* layouts timed by the sweep at create (output only) */
    double edge_iters_per_sec;   /* sweep rating of this layout, 0 when not timed (output only) */
} mwu_batch_layout;

/* Current layout of a batched handle.  MWU_ERR_STATE for a single-problem
 * handle, MWU_ERR_INVALID_ARG for NULL arguments. */
mwu_status mwu_batch_get_layout(void *s, mwu_batch_layout *out);

/* Replace the layout of a batched handle (the first four fields; the rest
 * are ignored).  Rebuilds the tile lists and the captured launch sequence;
 * results of later solves are those of the new layout (the same method, with
 * sums reduced in another order).  MWU_ERR_INVALID_ARG for values outside the
 * ranges above, MWU_ERR_STATE for a single-problem handle. */
mwu_status mwu_batch_set_layout(void *s, const mwu_batch_layout *layout);

/* Run the outer search (or the single fixed-lambda probe).
 * x_out: nullable, host, length = number of variables of the problem (batch:
 * the concatenation); receives x in the caller's variable order and scale.
 * objective_out, iterations_out: nullable, host (batch: length count).
 * info: nullable (batch: length count). */
mwu_status mwu_solve(void *s, double *x_out, double *objective_out, int64_t *iterations_out,
                     mwu_result_info *info);

/* Release every resource of the handle.  NULL is accepted. */
void mwu_destroy(void *s);

/* Static text for a status or error code. */
const char *mwu_status_string(mwu_status st);

/* Number of variables (columns) the handle exposes to the caller. */
int64_t mwu_num_variables(void *s);

/* ---------------------------------------------------------------------------
 * Probe-level access, used for per-pass comparisons and by the autograd
 * potential.  "param" is M for pure problems (the embedded objective row is
 * (1/M) 1^T), D (lambda) for MWU_MIXED.  Vectors are in the internal
 * (normalized, compacted) variable space of length mwu_probe_sizes().n.
 * ------------------------------------------------------------------------- */

typedef struct {
    int64_t n;        /* internal variables */
    int64_t m_P;      /* internal packing rows (1 for the embedded objective row) */
    int64_t m_C;      /* internal covering rows */
    double eta;       /* 10 ln(m_P + m_C) / eps (Algorithm 1) */
} mwu_sizes;

typedef struct {
    int32_t status;            /* MWU_PROBE_* */
    int64_t iterations;
    int64_t search_passes;
    double alpha;              /* last accepted step */
    double L_P, L_C;           /* smax(Px), smin(Cx) (Section 2.2) */
    double pack_bound, cover_bound;   /* weak-duality bounds seen so far */
    int64_t evaluations;       /* tests of Phi >= Psi, counted as a one-at-a-time Algorithm 3 makes them */
} mwu_probe_info;

mwu_status mwu_probe_sizes(void *s, mwu_sizes *out);

/* Start a probe at the given param.  x0 (host, nullable, length n): starting
 * point; NULL = the Algorithm 1 initial point eps / (n max_j P_ji). */
mwu_status mwu_probe_begin(void *s, double param, const double *x0);

/* Run max_iters more iterations of Algorithm 2 (fewer when the probe ends
 * first); a running probe pauses after exactly max_iters accepted steps.
 * forced_alpha (host, nullable, n_forced entries): use these steps instead
 * of the search for the next n_forced iterations (decision replay).  While
 * the probe is still running on return, its last accepted step is applied
 * by the next iteration's row pass: x, y and z read then are the iterate
 * before that step (mwu_probe_direction applies it first). */
mwu_status mwu_probe_run(void *s, int32_t max_iters, const double *forced_alpha, int32_t n_forced,
                         mwu_probe_info *info);

/* Compute g, h, d, P d, C d at the current x (after applying a pending
 * accepted step, see mwu_probe_run) without taking a new step.  The probe
 * then waits at the step search of this iteration: a later mwu_probe_run
 * continues there (first the stop tests of Algorithm 2 at this point), so
 * running, forming a direction and running again takes the same steps as
 * running alone.  MWU_ERR_STATE unless the probe is at an iteration start. */
mwu_status mwu_probe_direction(void *s);

/* Copy an internal vector to the host (double).  which: 0 x, 1 d, 2 g, 3 h,
 * 4 y = Px (m_P), 5 z = Cx (m_C), 6 dy = Pd (m_P), 7 dz = Cd (m_C), 8 the
 * accepted steps of the current probe (length = its iteration count).  len
 * must equal the vector's length.  g and h are those of the last
 * mwu_probe_direction call. */
mwu_status mwu_probe_read(void *s, int32_t which, double *out, int64_t len);

/* Evaluate Psi(alpha_k), Phi(alpha_k) (Section 4.1) and min(Cx + alpha_k Cd)
 * at the current x and direction, for k < count (count <= 16).  Outputs are
 * host arrays of length count; zmin_new is nullable.  Needs the direction of
 * mwu_probe_direction (MWU_ERR_STATE otherwise); changes no vector, so a
 * later mwu_probe_run continues as after mwu_probe_direction alone. */
mwu_status mwu_probe_eval_steps(void *s, const double *alphas, int32_t count, double *psi,
                                double *phi, double *zmin_new);

/* The Newton pass of MWU_STEP_NEWTON at one step alpha > 0: Psi(alpha),
 * Phi(alpha) and their derivatives Psi'(alpha), Phi'(alpha) (Section 4.2:
 * the averages of P d and C d under the weights of the moved point
 * Px + alpha Pd, Cx + alpha Cd), at the current x and direction.  Outputs
 * are host scalars.  Same state rules as mwu_probe_eval_steps. */
mwu_status mwu_probe_eval_newton(void *s, double alpha, double *psi, double *phi, double *dpsi,
                                 double *dphi);

/* Probe-level access to a batched handle: one probe of Algorithm 2 (with the
 * handle's step rule) on every instance at once, instance k at params[k] =
 * M_k (its objective row is (1/M_k) 1^T x, end of Section 2.2), started from
 * the Algorithm 1 point and run by the batched kernels in the handle's
 * layout.  A probe that is still running after max_iters accepted steps
 * pauses there (max_iters = 0: every probe runs to its outcome); calling
 * again starts new probes.  params: host, count entries, each > 0.  info:
 * host, count entries, nullable.  MWU_ERR_STATE on a single-problem handle,
 * MWU_ERR_INVALID_ARG for NULL params, max_iters < 0 or a parameter <= 0.
 * A later mwu_solve starts every outer search afresh. */
mwu_status mwu_batch_probe_run(void *s, const double *params, int32_t max_iters, mwu_probe_info *info);

/* A vector of instance `instance` after mwu_batch_probe_run, as
 * mwu_probe_read defines them: 0 x (the instance's edges, in its caller's
 * order), 1 d, 4 y = Px (its non-isolated vertices in vertex order), 6 dy =
 * Pd, 8 the accepted steps of its probe (len = its iteration count).  When a
 * probe paused, x is the iterate before its last accepted step and d the
 * direction formed at x.  MWU_ERR_STATE before any batched probe,
 * MWU_ERR_INVALID_ARG for an unknown vector, an instance out of range or a
 * length mismatch. */
mwu_status mwu_batch_probe_read(void *s, int32_t instance, int32_t which, double *out, int64_t len);

/* Time the main kernel of one pass of the iteration: which = 0 row /
 * transpose pass (the weights, their LSE totals and C^T u, P^T w), 1 column /
 * direction pass, 2 forward pass (P d, C d; a no-op in fused programs that
 * form it inside the search), 3 step-search pass over the exponential grid
 * (8 candidates from 1), 4 step-search pass over a bisection grid (15
 * candidates in [1, 2]), 5 the combined first pass of an iteration (the 8
 * exponential candidates and the 15 of the bisection of [2, 4]).  First the
 * pending accepted step is committed and one direction is formed at that
 * point; then the kernel is launched reps times on the handle's stream with
 * the probe state held (the finisher kernel of the pass is not launched),
 * timed with HIP events.  Afterwards the probe continues from the committed
 * point with a full iteration: the same iterate a run without the call
 * reaches, its LSE totals renormalized by a row pass with no step.  Outputs (host): average duration
 * in microseconds, algorithmic HBM bytes of one launch (every index, dense
 * vector and output counted once; nullable) and the nonzeros the pass visits
 * (nullable).  Needs a probe at an iteration start (mwu_probe_begin). */
mwu_status mwu_time_pass(void *s, int32_t which, int32_t reps, double *avg_us, double *bytes,
                         double *nnz);

/* ---------------------------------------------------------------------------
 * Smoothed potential for automatic differentiation: Phi(x) = smax_eta(P x) -
 * smin_eta(C x) at the handle's current param (Section 4.1) and its gradient
 * P^T grad smax(Px) - C^T grad smin(Cx) (the g - h of Algorithm 2).
 * x_dev, grad_dev: DEVICE pointers to double arrays of length n in the
 * internal variable space; stream: hipStream_t or NULL (handle stream).
 * ------------------------------------------------------------------------- */
mwu_status mwu_potential_forward(void *s, const double *x_dev, double *value_out, void *stream);
mwu_status mwu_potential_backward(void *s, const double *x_dev, double grad_scale, double *grad_dev,
                                  void *stream);

/* mwu_potential_backward for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same gradient, written to grad_dev as grad_scale (g - h),
 * with no allocation in the call.  Every reduction record and chunk partial
 * of its passes lives in a static device array of 8 MiB per GPU (held until
 * the process ends, shared by all calls on that GPU: calls that overlap on one
 * GPU race).  value_out (host, nullable) receives Phi(x) =
 * smax(Px) - smin(Cx), as mwu_potential_forward returns it.  Errors:
 * MWU_ERR_TOO_LARGE when the problem's records and chunk partials exceed the
 * array; MWU_ERR_STATE for programs without a potential (the fused vertex
 * cover), batch handles, or no probe begun; MWU_ERR_INVALID_ARG for NULL x_dev
 * or grad_dev. */
mwu_status mwu_potential_backward_noalloc(void *s, const double *x_dev, double grad_scale, double *grad_dev,
                                          double *value_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MWU_H */
