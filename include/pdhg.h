/*
 * pdhg.h -- C ABI of libpdhg.so, an MI355X (gfx950) implementation of the
 * restarted, diagonally preconditioned PDHG iteration for the standard-form LP
 *
 *     min c^T x   s.t.  A x = b,  x >= l      (l = 0 unless set)
 *     max b^T y + l^T z   s.t.  A^T y + z = c,  z >= 0
 *
 * (the primal/dual pair of Section 2 of Rothberg, "Concurrent Crossover for
 * PDHG", with an optional lower-bound vector used by iterative refinement).
 *
 * Conventions for every call:
 *  - Return value: PDHG_OK (0) or a negative pdhg_error; the message is in
 *    pdhg_last_error(ctx).  No C++ exception crosses this boundary.  Solver
 *    outcomes (converged, iteration limit, ...) are reported separately as a
 *    pdhg_status through an out-parameter.
 *  - `mem` says where caller pointers live: PDHG_MEM_HOST (pageable or pinned
 *    host memory) or PDHG_MEM_DEVICE (device memory of the context's GPU, for
 *    example a torch tensor's data_ptr()).  Device pointers are used only
 *    during the call and ordered on the context's stream; the call returns
 *    after the stream has finished with them.
 *  - Inputs are copied: the library owns its device copies, the caller may
 *    free or reuse its arrays when the call returns.  Output buffers belong
 *    to the caller and must hold the stated number of elements.
 *  - Index arrays: row pointers int64 (m+1 or n+1 entries, first 0, last nnz,
 *    non-decreasing), column indices int32 in [0, ncols), strictly increasing
 *    inside a row.  nnz must stay below 2^31.  Values are IEEE binary64.
 *  - A context is not thread-safe; only pdhg_cancel may be called from
 *    another thread while a call on the same context runs.
 *  - The library allocates its device buffers itself (hipMalloc) at load and
 *    configure time and frees them in pdhg_destroy.
 */
#ifndef PDHG_H
#define PDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdhg_ctx pdhg_ctx;
typedef struct pdhg_tape pdhg_tape;

/* Error codes: the call failed and changed nothing the caller relies on. */
enum pdhg_error {
    PDHG_OK = 0,
    PDHG_E_ARG = -1,        /* bad argument (null pointer, size, range) */
    PDHG_E_CSR = -2,        /* malformed CSR arrays */
    PDHG_E_TRANSPOSE = -3,  /* A^T is not the transpose of A (values bitwise) */
    PDHG_E_DEVICE = -4,     /* a HIP runtime call failed */
    PDHG_E_OOM = -5,        /* host or device allocation failed */
    PDHG_E_STATE = -6       /* call out of order (e.g. iterate before load) */
};

/* Solver status: the call succeeded; this says where the iteration stands. */
enum pdhg_status {
    PDHG_RUNNING = 0,
    PDHG_CONVERGED = 1,     /* maxresid <= eps_rel (Section 2 criteria) */
    PDHG_ITER_LIMIT = 2,
    PDHG_TIME_LIMIT = 3,
    PDHG_CANCELLED = 4,
    PDHG_NUMERICAL = 5      /* a KKT quantity became NaN or infinite */
};

enum { PDHG_MEM_HOST = 0, PDHG_MEM_DEVICE = 1 };

/* Arithmetic of the bulk iteration (SpMVs and fused vector updates).  The
 * KKT reductions, restart decisions and refinement update are FP64 always. */
enum { PDHG_FP64 = 0, PDHG_FP32 = 1 };

/*
 * Solver parameters.  The paper fixes the stopping rule (the three relative
 * inequalities of Section 2) and the snapshot schedule (Algorithm 1,
 * Section 3.1: a snapshot whenever maxresid <= eps_target, then a tenfold
 * smaller target, until eps_rel).  It states no PDHG internals; the defaults
 * of the remaining fields are the published PDLP-style choices.
 */
typedef struct {
    int32_t precision;          /* PDHG_FP64 (default) or PDHG_FP32 */
    int32_t ruiz_passes;        /* Ruiz l_inf equilibration passes (10) */
    int32_t power_iters;        /* power-iteration steps for ||A~||_2 (100) */
    int32_t eval_every;         /* iterations between KKT evaluations (64) */
    int32_t literal_snapshots;  /* 1: at most one level per evaluation, as
                                   Algorithm 1 checks one target at a time */
    int32_t n_levels;           /* number of snapshot tolerances (<= 32) */
    const double *levels;       /* strictly descending, copied at configure */
    double eps_rel;             /* stop when maxresid <= eps_rel (1e-6) */
    double eta;                 /* step size; <= 0: eta_factor / sigma_hat */
    double omega0;              /* initial primal weight; <= 0: ||c~||/||b~|| */
    double eta_factor;          /* 0.9 */
    double beta_suff;           /* restart if KKT <= beta_suff * KKT_last (0.2) */
    double beta_nec;            /* ... or <= beta_nec * KKT_last and rising (0.8) */
    double beta_art;            /* ... or t >= beta_art * k (0.36) */
    double omega_theta;         /* primal-weight smoothing (0.5) */
    int64_t max_iters;          /* total iteration limit */
    double time_limit_s;        /* wall-clock limit per solve (3600) */
    int32_t use_graph;          /* replay eval_every-iteration batches as hipGraphs */
    int32_t variant;            /* 0: averaged iterates (PDLP-style restarts);
                                   1: reflected Halpern iteration (cuPDLP+-style) */
    double reflect;             /* Halpern reflection rho in [0, 1] (1) */
    int32_t omega_rule;         /* primal weight at a restart, from the
                                   distances dx, dy travelled since the last
                                   one: 0 smoothing, log w += theta (log(dy/dx)
                                   - log w); 1 PID on e = log(w dx / dy):
                                   log w -= kp e + ki sum(e) + kd (e - e_prev) */
    int32_t pad_;
    double pid_kp, pid_ki, pid_kd;  /* PID gains (0.99, 0.01, 0) */
    int32_t stop_on;            /* what the eps_rel stop and the candidate
                                   choice measure: 0 maxresid (default),
                                   1 rel_p only, 2 rel_d only (feasibility) */
    int32_t polish;             /* 1: feasibility polishing (see
                                   pdhg_iterate) */
    double polish_frac;         /* polishing phase budget as a fraction of
                                   the iterations so far (0.125) */
} pdhg_params;

/* Relative KKT errors of an unscaled iterate on the original data:
 * rel_p = ||b - Ax||_2 / (1 + ||b||_2), rel_d = ||r_D||_2 / (1 + ||c||_2)
 * with z = max(0, c - A^T y) and r_D = A^T y + z - c, rel_gap =
 * |pobj - dobj| / (1 + |pobj| + |dobj|), maxresid = max of the three
 * (Section 2's three inequalities; maxresid of Algorithm 1). */
typedef struct {
    double rel_p, rel_d, rel_gap, maxresid;
    double pobj, dobj;          /* c^T x and b^T y + l^T z */
    double norm_rp, norm_rd;    /* ||r_P||_2, ||r_D||_2 */
    double rp_inf, rd_inf;      /* max-norms (informational) */
    int64_t iter;
    int32_t candidate;          /* 0 current iterate, 1 average */
    int32_t pad_;
} pdhg_kkt;

typedef struct {
    int32_t status, candidate;  /* pdhg_status; returned candidate (0 current,
                                   1 average or T(z), 2 polished pair) */
    int64_t iters;
    int32_t restarts, n_snap;
    double sigma_hat, eta, omega0, omega, tau, sigma;
    double t_setup, t_iter;     /* seconds in configure / in iterate calls */
    pdhg_kkt kkt;               /* of the iterate get_iterate returns */
    int32_t polish_attempts;    /* feasibility polishing attempts */
    int32_t pad_;
    int64_t polish_iters;       /* iterations spent in polishing phases */
} pdhg_info;

typedef struct {
    double level;               /* tolerance that fired */
    int64_t iter;               /* iteration of the emitting evaluation */
    double maxresid;            /* maxresid of the emitted iterate */
    int32_t candidate, pad_;
    double t_wall;              /* seconds since the solve started */
} pdhg_snapshot_info;

typedef struct {
    double outer_eps;           /* stop when FP64 maxresid <= outer_eps (1e-8) */
    double inner_eps;           /* inner (correction LP) eps_rel (1e-4) */
    int32_t max_rounds;         /* refinement rounds after round 0 (8) */
    int32_t cap_log2;           /* scale growth cap per round, 2^cap (10) */
    int64_t max_inner_iters;    /* iteration budget of a round's inner solve
                                   (200000); see pdhg_solve_refined */
    double progress;            /* an inner solve also stops once the refined
                                   point's FP64 maxresid <= max(outer_eps,
                                   progress * maxresid before the round) (1e-2) */
    int32_t inner_precision;    /* PDHG_FP32 (default) or PDHG_FP64 inner solves */
    int32_t omega_carry;        /* 1: a round starts from the final primal
                                   weight of round 0 or of the last later
                                   round whose inner solve converged, times
                                   (D_D/D_D,then) / (D_P/D_P,then); 0: from
                                   ||c^||/||b^|| of the correction LP (1) */
    int64_t stall_iters;        /* a round ends early once the refined point
                                   has not improved for max(stall_iters, 4 x
                                   the iterations it took to reach its best)
                                   inner iterations; 0: 65536 (the default),
                                   < 0: never; see pdhg_solve_refined */
} pdhg_refine_params;

typedef struct {
    int32_t status, rounds;
    int64_t inner_iters;        /* summed over rounds */
    double t_total;             /* seconds */
    pdhg_kkt kkt;               /* FP64 KKT of the final iterate */
} pdhg_refine_info;

/* Per-kernel timing record (HIP events around each launch, when enabled). */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} pdhg_kernel_time;

/* ---- host-only calls (no GPU needed) ---------------------------------- */

/* Fill *p with the defaults listed above (precision FP64, eps_rel 1e-6,
 * no snapshot levels, max_iters 2^62, use_graph 1). */
int pdhg_params_default(pdhg_params *p);
int pdhg_refine_params_default(pdhg_refine_params *p);

/* Algorithm 1's targets (Section 3.1): eps_cross / 10^j for every j with a
 * value above eps_rel, followed by eps_rel itself.  Writes at most cap
 * values to out and returns how many, or a negative error. */
int pdhg_alg1_levels(double eps_cross, double eps_rel, double *out, int cap);

/* Check one CSR matrix with `rows` rows over `cols` columns: rp[0] = 0,
 * rp[rows] = nnz, non-decreasing, 0 <= ci < cols, strictly increasing inside
 * each row, nnz < 2^31.  Returns PDHG_OK or PDHG_E_CSR with a message in msg
 * (msg may be NULL). */
int pdhg_validate_csr(int64_t rows, int64_t cols, int64_t nnz,
                      const int64_t *rp, const int32_t *ci, char *msg,
                      int msg_len);

/* Check that (at_rp, at_ci, at_v) is exactly the transpose of
 * (a_rp, a_ci, a_v), values compared bitwise.  If perm is not NULL, write
 * perm[p] = position in A^T's arrays of A's nonzero p.  Returns PDHG_OK,
 * PDHG_E_CSR or PDHG_E_TRANSPOSE. */
int pdhg_check_transpose(int64_t m, int64_t n, int64_t nnz,
                         const int64_t *a_rp, const int32_t *a_ci,
                         const double *a_v, const int64_t *at_rp,
                         const int32_t *at_ci, const double *at_v,
                         int64_t *perm, char *msg, int msg_len);

/* Row-length bins of one CSR matrix (rows+1 int64 row pointers) for a tile
 * of `tile` nonzeros: writes up to cap descriptors of 4 int32 each
 * (first row, end row, part, number of parts) in launch order and returns
 * the number of descriptors (or a negative error).  Rows longer than
 * split_threshold are split into parts of split_chunk nonzeros.  Host only;
 * the library calls the same planner at load time, where it also caps a
 * multi-row block at 256 rows (tuning key "block_rows"); this entry point
 * applies the tile cap alone. */
int pdhg_plan_bins(int64_t rows, const int64_t *rp, int tile,
                   int64_t split_threshold, int64_t split_chunk,
                   int32_t *out, int64_t cap);

/* ---- context lifecycle ------------------------------------------------- */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * to launch on (for example torch.cuda.current_stream().cuda_stream) or NULL
 * for a stream the context creates (default priority). */
int pdhg_create(int device, void *hip_stream, pdhg_ctx **out);
void pdhg_destroy(pdhg_ctx *ctx);
/* Last error message of this context; valid until the next call on it.
 * With ctx NULL: the message of this thread's last failed pdhg_create. */
const char *pdhg_last_error(const pdhg_ctx *ctx);

/* ---- problem data ------------------------------------------------------ */

/* Load the data of Section 2's primal problem min c^T x, Ax = b, x >= 0
 * (with x >= lb when lb is given): CSR A (m x n) and its explicit transpose
 * CSR A^T (n x m), b (m), c (n) and optional lower bounds lb (n; NULL = 0).
 * Validates both CSRs and the transpose relation (PDHG_E_CSR /
 * PDHG_E_TRANSPOSE), then builds the row-length bins of both matrices.
 * Replaces any earlier problem (and invalidates its adjoint tapes). */
int pdhg_load(pdhg_ctx *ctx, int64_t m, int64_t n, int64_t nnz,
              const int64_t *a_rp, const int32_t *a_ci, const double *a_v,
              const int64_t *at_rp, const int32_t *at_ci, const double *at_v,
              const double *b, const double *c, const double *lb, int mem);

/* Replace A's values (nnz, in A's CSR order); A^T follows through the load
 * permutation.  The scaling factors of the last configure are kept (frozen)
 * and re-applied; call pdhg_configure to recompute them. */
int pdhg_set_values(pdhg_ctx *ctx, const double *a_v, int mem);
/* Replace b (m) and c (n) (either may be NULL to keep it); frozen scaling. */
int pdhg_set_rhs_obj(pdhg_ctx *ctx, const double *b, const double *c, int mem);

/* ---- solve ------------------------------------------------------------- */

/* Copy the parameters and snapshot levels, compute the Ruiz factors D_r, D_c
 * (ruiz_passes passes), the scaled data A~ = D_r A D_c, b~ = D_r b,
 * c~ = D_c c, l~ = l / D_c, the power-iteration estimate sigma_hat of
 * ||A~||_2, the step size eta, the primal weight omega and tau = eta / omega,
 * sigma = eta * omega, and reset the iterate to zero and the status to
 * RUNNING.  Required before pdhg_iterate. */
int pdhg_configure(pdhg_ctx *ctx, const pdhg_params *p);

/* Warm start from unscaled x (n) and y (m) (either may be NULL = zero);
 * resets the averages, the restart state and the status.  The paper's
 * Algorithm 1 starts PDHG from a given iterate (its input); this sets it.
 * With no call the iteration starts from zero. */
int pdhg_set_iterate(pdhg_ctx *ctx, const double *x, const double *y, int mem);

/* Run up to max_iters more iterations (the parameter max_iters bounds the
 * total).  One iteration is the fused primal step
 *   x <- max(l~, x - tau (c~ - A~^T y))
 * followed by the extrapolated dual step
 *   y <- y + sigma (b~ - (2 A~ x_new - A~ x_old)),
 * and the uniform averages since the last restart.  Every eval_every
 * iterations (and once before the first) the current and averaged iterates
 * are evaluated in FP64; a snapshot is emitted for each not-yet-emitted
 * level >= the better candidate's maxresid (Algorithm 1's test), the solve
 * stops when it is <= eps_rel, and otherwise the adaptive restart rule runs.
 * Returns when the status leaves RUNNING or the iterations are done; *status
 * receives the pdhg_status.
 * With variant = 1 an iteration instead forms T(z) (the same fused steps) and
 * z <- lambda((1 + rho)T(z) - rho z) + (1 - lambda) z_0, lambda = t/(t+1) for
 * the t-th step since the restart point z_0; the evaluations use T(z) as the
 * candidate (z itself is not projected), restarts test ||z - T(z)||_omega and
 * restart at T(z), and a stopped solve reports T(z).
 * With polish = 1 (feasibility polishing, the procedure the paper's closing
 * discussion cites): at an evaluation (k > 0) that does not stop, whose
 * candidate has rel_gap <= eps_rel, and once k has reached the next
 * polishing point (initially 0), the candidate is set aside before the
 * restart test; after it, a primal phase (same variant, step size and primal
 * weight) solves min 0 s.t. Ax = b, x >= l from (candidate x, 0) until rel_p
 * <= eps_rel, and a dual phase solves min c^T x s.t. Ax = 0, x >= 0 from
 * (0, candidate y) until rel_d <= eps_rel, each within max(eval_every,
 * ceil(polish_frac k / eval_every) eval_every) iterations.  If both succeed
 * and the pair has maxresid <= eps_rel the solve stops with it (candidate 2);
 * otherwise the main iteration continues unchanged and the next polishing
 * point is 2k. */
int pdhg_iterate(pdhg_ctx *ctx, int64_t max_iters, int *status);

/* Ask a running pdhg_iterate / pdhg_solve_refined to stop at its next
 * evaluation check with PDHG_CANCELLED.  Thread-safe and idempotent.  This is
 * Algorithm 1's termination of the PDHG run once a crossover thread has found
 * the optimal basis first (Section 3.1); the concurrent-crossover calls below
 * use it for that, and a caller running its own crossover threads may too. */
int pdhg_cancel(pdhg_ctx *ctx);

/* Counters, step sizes and the KKT of the current iterate. */
int pdhg_get_info(pdhg_ctx *ctx, pdhg_info *out);

/* FP64 relative KKT errors (Section 2's three relative quantities on the
 * unscaled problem, and their maximum, Algorithm 1's maxresid) of: which =
 * 0 current iterate, 1 average
 * (valid after at least one iteration since the last restart; for the
 * Halpern variant T(z) of the last evaluation), 2 the better of the two by
 * maxresid (a tie goes to the current iterate); out->candidate says which. */
int pdhg_residuals(pdhg_ctx *ctx, int which, pdhg_kkt *out);

/* Unscaled current iterate: the primal x (n) and dual y (m) of Section 2's
 * pair, and the dual slack z = max(0, c - A^T y) (n), which the paper leaves
 * implicit for a PDHG iterate; with it, r_D = A^T y + z - c.  Any pointer
 * may be NULL. */
int pdhg_get_iterate(pdhg_ctx *ctx, double *x, double *y, double *z, int mem);

/* Ruiz factors of the last configure: dr (m), dc (n). */
int pdhg_get_scaling(pdhg_ctx *ctx, double *dr, double *dc, int mem);

/* Evaluation log: up to cap records of 8 doubles (iteration, maxresid of
 * current and average, KKT_omega of current and average, restarted flag,
 * restart candidate, omega after the evaluation).  *count gets the total. */
int pdhg_eval_log(pdhg_ctx *ctx, double *out, int cap, int *count);

/* ---- snapshots (Algorithm 1's crossover starting points) --------------- */

/* Number of snapshots emitted since the last configure (or refinement). */
int pdhg_snapshot_count(pdhg_ctx *ctx, int *count);
/* Copy snapshot idx (0-based, in emission order): info plus unscaled
 * x (n), y (m), z (n); any pointer may be NULL.  A snapshot is an iterate
 * Algorithm 1 (Section 3.1) hands to a crossover thread, taken when the
 * better candidate's maxresid first reaches a level; its z = max(0, c -
 * A^T y) is the dual slack of Section 2's dual problem. */
int pdhg_snapshot(pdhg_ctx *ctx, int idx, pdhg_snapshot_info *info,
                  double *x, double *y, double *z, int mem);
/* Snapshot notification: Algorithm 1's hand-over of an iterate to a CPU
 * crossover thread (Section 3.1; the paper pulls the iterate from the GPU to
 * the CPU for this).  Called on one library thread, in emission order, once
 * the snapshot's copy to pinned host memory is complete, with the snapshot
 * index, its info and its unscaled x (n), y (m), z (n) in that host copy.
 * The pointers are valid only during the call (copy what is kept); a later
 * emission of the same level waits until the call has returned.  cb must not
 * call into the context. */
typedef void (*pdhg_snapshot_cb)(void *user, int idx,
                                 const pdhg_snapshot_info *info,
                                 const double *x, const double *y,
                                 const double *z);
/* Register cb (NULL: none) for the snapshots of later iterate / refinement
 * calls on this context. */
int pdhg_set_snapshot_callback(pdhg_ctx *ctx, pdhg_snapshot_cb cb, void *user);

/* ---- Algorithm 1: concurrent crossover ---------------------------------- */

/* A crossover routine supplied by the caller (the paper's CPU crossover, which
 * this library does not implement).  Called on a library thread with a
 * snapshot's unscaled x (n), y (m), z (n) (valid for the duration of the
 * call) and `cancel`, which becomes nonzero once another thread has won; the
 * library writes it with an atomic store, and the routine should poll it
 * (a volatile or atomic 32-bit load) and return promptly.  Returns 1 if it
 * found a basic optimal solution, 0 otherwise.  idx is the snapshot index, or
 * -1 for the final iterate. */
typedef int (*pdhg_crossover_fn)(void *user, int idx,
                                 const pdhg_snapshot_info *info,
                                 const double *x, const double *y,
                                 const double *z,
                                 const volatile int32_t *cancel);

/* Concurrent crossover PDHG (Algorithm 1, Section 3.1): iterate; every
 * snapshot the configured levels emit (for the paper's schedule, configure
 * with pdhg_alg1_levels(eps_cross, eps_rel)) launches `fn` on a new host
 * thread, at most max_threads at a time (0 means no limit).  A snapshot that
 * finds every thread busy is copied to the host and queued, and starts when
 * a thread returns; PDHG keeps iterating meanwhile, as Algorithm 1's loop
 * does while its crossover threads run.  The first call to return 1 wins: the others see
 * *cancel set, PDHG is stopped, and *winner receives its index.  When PDHG
 * reaches eps_rel without a winner, `fn` also runs on the calling thread from
 * the final iterate (idx -1) unless a snapshot was taken from that same
 * iterate.  *winner is -2 if no call succeeded.  *status receives the PDHG
 * status (PDHG_CANCELLED when a crossover won first).  A pdhg_cancel from
 * another thread during the call stops PDHG and sets *cancel for the
 * crossovers too; a cancel requested before the call is dropped.  Returns
 * after every crossover thread has finished. */
int pdhg_concurrent_crossover(pdhg_ctx *ctx, pdhg_crossover_fn fn, void *user,
                              int max_threads, int64_t max_iters,
                              int *winner, int *status);

/* Algorithm 1 over FP32 bulk iterations with FP64 refinement: as
 * pdhg_concurrent_crossover, with pdhg_solve_refined(ctx, rp, info) (rp NULL:
 * defaults) as the solve, whose snapshots of the refined iterate launch the
 * crossovers; a winner stops the refinement (*status PDHG_CANCELLED). */
int pdhg_concurrent_crossover_refined(pdhg_ctx *ctx, pdhg_crossover_fn fn,
                                      void *user, int max_threads,
                                      const pdhg_refine_params *rp,
                                      int *winner, int *status,
                                      pdhg_refine_info *info);

/* ---- FP32 bulk iteration with FP64 refinement --------------------------- */

/* Iterative refinement: round 0 solves the LP with the bulk iteration in
 * FP32; each later round computes FP64 residuals r_P = b - Ax,
 * d = c - A^T y, power-of-two scales Delta_P, Delta_D, solves the correction
 * LP  min (Delta_D d)^T xh  s.t.  A xh = Delta_P r_P,  xh >= -Delta_P x
 * with FP32 bulk iterations and FP64 evaluations, and updates in FP64
 * x <- max(0, x + xh / Delta_P), y <- y + yh / Delta_D, until the FP64
 * maxresid <= outer_eps.  Each inner evaluation measures the refined point
 * in FP64 and keeps the best one.  An inner solve stops at inner_eps, when
 * the refined point has gained the factor `progress`, when it has not
 * improved for max(stall_iters, 4 x the iterations to its best), or at its
 * budget of max_inner_iters; a budget or stall end before any improvement
 * extends the same solve, doubling budget and stall window, up to 16 times
 * max_inner_iters.  The round then takes its best refined point (or the
 * final one, if better) when that improves on the maxresid before the round:
 * partial progress is kept.  A round that cannot improve ends the refinement
 * (status PDHG_ITER_LIMIT).  With omega_carry, a round after the first starts
 * from the final primal weight of round 0 or of the last later round whose
 * inner solve converged, rescaled by the change of Delta_D / Delta_P since
 * then.
 * Uses the parameters of the last configure (its
 * precision field is ignored; its time_limit_s bounds the whole
 * refinement).  The configured snapshot levels apply to the refined iterate:
 * its FP64 maxresid is measured before every round and at the end, and
 * every level it has reached emits a snapshot of it (iter = inner iterations
 * so far; candidate 0), with the snapshot callback if one is set.  The
 * refined iterate becomes the context's current iterate. */
int pdhg_solve_refined(pdhg_ctx *ctx, const pdhg_refine_params *rp,
                       pdhg_refine_info *info);

/* Per-round log of the last pdhg_solve_refined: up to cap records of 10
 * doubles (round, FP64 maxresid of the outer iterate before the round,
 * Delta_P, Delta_D, inner iterations, inner status, inner maxresid, seconds
 * since the start, 1 if the round was ended early for stalling, 1 if its
 * refined point was accepted); *count gets the number of records. */
int pdhg_refine_log(pdhg_ctx *ctx, double *out, int cap, int *count);

/* ---- unrolled steps and their adjoint ------------------------------------ */

/* Run K plain PDHG steps (no restarts, no averaging) on the configured,
 * scaled problem with fixed tau, sigma, from unscaled (x0, y0) (NULL: zero),
 * in `precision`; write unscaled x_K (n).  Stores (x, y, A~x) every
 * ckpt_every steps in a new tape (*tape; free with pdhg_tape_free). */
int pdhg_unrolled_forward(pdhg_ctx *ctx, int K, int ckpt_every,
                          int precision, double tau, double sigma,
                          const double *x0, const double *y0, double *xK,
                          int mem, pdhg_tape **tape);
/* Reverse pass for the loss gradient gxK = dL/dx_K (n, unscaled): writes
 * dL/dc (n), dL/db (m) and dL/dA.values (nnz, A's CSR order), with the
 * scaling factors held fixed.  Segments between checkpoints are recomputed
 * with the forward kernels, which are deterministic, so the result does not
 * depend on ckpt_every.  The projection's subgradient is 0 at a tie.
 * The replay reads the context's current problem data, so a tape is valid
 * only until the next pdhg_load, pdhg_configure, pdhg_set_values or
 * pdhg_set_rhs_obj (with data) on its context: after any of them this call
 * returns PDHG_E_STATE (a reload also frees the tape's device memory at
 * once; the handle still needs pdhg_tape_free). */
int pdhg_unrolled_backward(pdhg_tape *tape, const double *gxK, double *gc,
                           double *gb, double *gAval, int mem);
/* Release a tape.  pdhg_destroy releases the device memory of the tapes of
 * its context; their handles must still be passed to pdhg_tape_free, and
 * pdhg_unrolled_backward on them returns PDHG_E_STATE. */
void pdhg_tape_free(pdhg_tape *tape);

/* ---- the CPU platform (host only) ---------------------------------------- */

/* K plain PDHG steps on the host's cores (the paper's multi-threaded CPU
 * PDHG, Section 4.1; its bandwidth remark, Section 5): with `threads`
 * threads, each owning a contiguous range of rows of equal nonzero count,
 *   x <- max(0, x - tau (c - A^T y))   over the rows of A^T (at_*),
 *   y <- y + sigma (b - A (2 x_new - x_old))   over the rows of A (a_*),
 * a barrier between the halves.  The matrices are used as given (pass the
 * scaled ones for scaled steps); x (n) and y (m) are updated in place;
 * *seconds (may be NULL) receives the wall time of the K steps.  No GPU is
 * used.  Returns PDHG_OK, PDHG_E_ARG or PDHG_E_OOM. */
int pdhg_cpu_steps(int64_t m, int64_t n, const int64_t *a_rp,
                   const int32_t *a_ci, const double *a_v,
                   const int64_t *at_rp, const int32_t *at_ci,
                   const double *at_v, const double *b, const double *c,
                   double tau, double sigma, int K, int threads, double *x,
                   double *y, double *seconds);

/* ---- the CPU PDHG (host only) --------------------------------------------- */

/* The restarted PDHG on the host's cores: the paper's CPU platform (Section
 * 4.1 runs its PDHG on CPU cores next to the GPU one; Section 5 remarks that a
 * fraction of the cores saturates the CPU's memory bandwidth).  The method is
 * the GPU path's, in FP64 only: Ruiz equilibration, the power-iteration step
 * size, the averaged or the reflected Halpern iteration, the FP64 KKT
 * evaluation every eval_every iterations with the same snapshot, stop,
 * restart and primal-weight decisions (Section 2's criteria, Algorithm 1's
 * snapshot test).  Feasibility polishing, FP32 and graphs are GPU-only.  Work
 * is split over a pool of `threads` host threads: the primal half over row
 * ranges of A^T, the dual half over row ranges of A, each holding an equal
 * share of the nonzeros; reductions are summed over fixed chunks of 4096 rows
 * in chunk order, so the results do not depend on the thread count.  No GPU is
 * used.  Every pointer is host memory; conventions as for the GPU calls (a
 * context is not thread-safe except pdhg_cpu_cancel; inputs are copied). */
typedef struct pdhg_cpu pdhg_cpu;
int pdhg_cpu_create(int threads, pdhg_cpu **out);
void pdhg_cpu_destroy(pdhg_cpu *ctx);
const char *pdhg_cpu_last_error(const pdhg_cpu *ctx);
/* Replace the thread pool (1 .. 1024 threads); the problem and iterate stay. */
int pdhg_cpu_set_threads(pdhg_cpu *ctx, int threads);
/* As pdhg_load (Section 2's primal problem; A^T must be A's exact
 * transpose), host arrays only. */
int pdhg_cpu_load(pdhg_cpu *ctx, int64_t m, int64_t n, int64_t nnz,
                  const int64_t *a_rp, const int32_t *a_ci, const double *a_v,
                  const int64_t *at_rp, const int32_t *at_ci,
                  const double *at_v, const double *b, const double *c,
                  const double *lb);
/* As pdhg_configure; precision must be PDHG_FP64 and polish 0 (PDHG_E_ARG
 * otherwise); use_graph is ignored.  Resets the iterate to zero. */
int pdhg_cpu_configure(pdhg_cpu *ctx, const pdhg_params *p);
/* As pdhg_iterate: up to max_iters more iterations, the evaluation at k = 0
 * and every eval_every iterations; *status receives the pdhg_status. */
int pdhg_cpu_iterate(pdhg_cpu *ctx, int64_t max_iters, int *status);
int pdhg_cpu_cancel(pdhg_cpu *ctx);
/* As pdhg_get_info; kkt is recomputed for the current iterate. */
int pdhg_cpu_get_info(pdhg_cpu *ctx, pdhg_info *out);
/* Unscaled current iterate x (n), y (m), z = max(0, c - A^T y) (n); any
 * pointer may be NULL. */
int pdhg_cpu_get_iterate(pdhg_cpu *ctx, double *x, double *y, double *z);
int pdhg_cpu_get_scaling(pdhg_cpu *ctx, double *dr, double *dc);
/* As pdhg_eval_log (8 doubles per evaluation). */
int pdhg_cpu_eval_log(pdhg_cpu *ctx, double *out, int cap, int *count);
int pdhg_cpu_snapshot_count(pdhg_cpu *ctx, int *count);
int pdhg_cpu_snapshot(pdhg_cpu *ctx, int idx, pdhg_snapshot_info *info,
                      double *x, double *y, double *z);
/* Streaming read bandwidth of the host with `threads` threads: `reps` sums
 * over an array of `bytes` bytes (first touched by the thread that reads each
 * part), after one warm-up pass; *gb_s = bytes reps / time / 1e9.  The
 * ceiling the CPU PDHG's iteration rate is compared with. */
int pdhg_cpu_stream_bw(int threads, int64_t bytes, int reps, double *gb_s);

/* ---- kernels for checking and measurement ------------------------------ */

/* One binned SpMV on the device: which = 0: out (m) = A in (n);
 * which = 1: out (n) = A^T in (m).  scaled = 1 uses A~, 0 the loaded A.
 * precision selects the FP64 or the FP32 kernel (FP32 rounds `in` and the
 * values to float and accumulates in float; out is widened to double). */
int pdhg_spmv(pdhg_ctx *ctx, int which, int scaled, int precision,
              const double *in, double *out, int mem);

/* Allocation-free variant of pdhg_spmv, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * pdhg_spmv (bitwise); its staging vectors (input and output in the internal
 * order, plus their FP32 copies for precision = PDHG_FP32) live in a
 * library-owned device array of PDHG_SPMV_NOALLOC_MAX_BYTES bytes, one per
 * GPU, held from library load until the process ends, instead of buffers
 * allocated per call.  The call itself allocates nothing on the device or
 * the host.  Staging needs 8 (rows + cols) bytes in FP64 and 12 (rows + cols)
 * bytes in FP32 (each array rounded up to 256 bytes), rows x cols being the
 * side's shape (A: m x n, A^T: n x m); larger problems get PDHG_E_ARG and a
 * message.  Every context on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (from several threads, or on several streams)
 * race and must be serialised by the caller.  The array keeps the last
 * call's contents; nothing in it needs to start at zero.  With
 * mem = PDHG_MEM_DEVICE the call issues only kernels and device-to-device
 * copies on the context's stream, followed by a stream synchronisation. */
#define PDHG_SPMV_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int pdhg_spmv_noalloc(pdhg_ctx *ctx, int which, int scaled, int precision,
                      const double *in, double *out, int mem);

/* Row-bin tuning, taking effect at the next pdhg_load:
 *  "split_threshold": nnz above which a row is split over several
 *      workgroups; "split_chunk": nnz per split part;
 *  "panels_a", "panels_at": column panels (1, 2, 4 or 8; 0 = chosen from
 *      the sizes, the default) of A (the table x the dual step gathers) and
 *      of A^T (the table y the primal step gathers).  With P > 1 panels an
 *      SpMV side runs as P column panels, each on the workgroups of 8 / P of
 *      the 8 XCDs, so that each XCD's L2 holds its panel's part of the
 *      table; rows are summed over the panels in panel order, so results stay
 *      deterministic but round differently from P = 1;
 *  "stream_nt": 1 streams the CSR arrays with non-temporal loads, 0 with
 *      plain loads, -1 (default) chooses per side: non-temporal when the
 *      FP64 gather table per XCD (8 cols / P bytes) exceeds 3 MiB;
 *  "sort_rows", "sort_cols": internal order of A's rows / columns: 1 sorts
 *      them by decreasing length, 0 keeps the given order, -1 (default)
 *      sorts a dimension only when its longest line exceeds 8 times the
 *      mean.  Results round differently with another order, and the
 *      reported iterates stay in the caller's order either way;
 *  "block_rows": at most this many rows per multi-row block (default 256,
 *      one per lane of a workgroup; 0 leaves the cap at the tile's nonzero
 *      count).
 * Returns PDHG_E_ARG for an unknown key or a value out of range. */
int pdhg_set_tuning(pdhg_ctx *ctx, const char *key, int64_t value);
/* Row-block statistics of matrix which (0 = A, 1 = A^T): counts of blocks
 * by kind {multi-row, single-row, split parts} in out[0..2]. */
int pdhg_bin_stats(pdhg_ctx *ctx, int which, int64_t *out3);
/* Host-only: the number of column panels (1, 2, 4 or 8) pdhg_load chooses
 * for an SpMV side of `rows` rows, nnz nonzeros and a gather table of `cols`
 * FP64 entries, or a negative error code. */
int pdhg_choose_panels(int64_t rows, int64_t cols, int64_t nnz);
/* Host-only: the column-panel layout pdhg_load builds for a CSR (rows x cols,
 * int64 row pointers rp, columns ci sorted within each row) cut at
 * cut[0] = 0 <= cut[1] <= ... <= cut[P] = cols, P in {1, 2, 4, 8}.
 * srp (P*rows+1) receives the stacked matrix's row pointers: stacked row
 * p*rows+i holds row i's entries with column in [cut[p], cut[p+1]); src
 * (nnz) the position in rp/ci of each stacked entry.  The row blocks for
 * tile `tile` (no splits) are written to out as (r0, r1, part, nparts), up
 * to cap blocks, in launch order: block w runs on XCD w % 8, which serves
 * panel (w % 8) % P; r0 == r1 marks padding.  Returns the number of blocks,
 * or a negative error code (PDHG_E_ARG also when P * rows >= 2^31: stacked
 * rows are indexed in int32, and pdhg_load halves P until they fit). */
int pdhg_plan_panels(int64_t rows, int64_t cols, const int64_t *rp,
                     const int32_t *ci, int P, const int64_t *cut, int tile,
                     int64_t *srp, int32_t *src, int32_t *out, int64_t cap);
/* Number of column panels in use for matrix which (0 = A, 1 = A^T) of the
 * loaded problem, in *panels. */
int pdhg_panel_count(pdhg_ctx *ctx, int which, int *panels);

/* Random-gather rate of this GPU (measurement only; needs a context, not a
 * problem).  One kernel streams n_gathers (index, value) pairs in the
 * precision's value type, 4096 pairs per workgroup, with the SpMV's 16-byte
 * loads (non-temporal when stream_nt = 1), gathers table[index] for each
 * from a table of table_entries values and sums the products.  Workgroup w
 * draws its indices uniformly at random (a fixed counter-based hash) from
 * panel (w % 8) % panels of the table, the slice that the XCD it runs on
 * gathers from in a panelled SpMV side.  After one warm-up launch, reps
 * launches are timed with HIP events on the context's stream;
 * *gathers_per_s = n_gathers reps / time.  This is the ceiling against which
 * the step kernels' gathers are measured: the SpMVs make one random gather
 * per nonzero, which the algorithmic byte count prices as 8 bytes but the
 * memory system serves a cache line at a time.  Allocates and frees its
 * buffers (about 12 n_gathers + 8 table_entries bytes in FP64). */
int pdhg_gather_probe(pdhg_ctx *ctx, int64_t table_entries, int precision,
                      int panels, int stream_nt, int64_t n_gathers, int reps,
                      double *gathers_per_s);

/* Enable (1) or disable (0) HIP-event timing of every iteration-kernel
 * launch (batches then run without graphs).  pdhg_kernel_times fills up to
 * cap records and sets *count; reset clears the records. */
int pdhg_profile(pdhg_ctx *ctx, int enable);
int pdhg_kernel_times(pdhg_ctx *ctx, pdhg_kernel_time *out, int cap,
                      int *count, int reset);

#ifdef __cplusplus
}
#endif
#endif /* PDHG_H */
