/*
 * pdhg_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, slow and deliberately obvious FP64 CPU implementation of
 * the restarted, diagonally preconditioned PDHG iteration for the
 * standard-form LP   min c^T x  s.t.  A x = b,  x >= l  (l = 0 unless given),
 * used to check the HIP library.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or helper with the HIP path: it reads A through its CSR only (products with
 * A^T are formed by scattering over A's rows) and works on the original data
 * wherever the paper's definitions do.
 *
 * What is fixed by the paper (Rothberg, "Concurrent Crossover for PDHG"):
 *   - the primal/dual pair and the residuals r_P = b - Ax, r_D = A^T y + z - c
 *     (Section 2, the displayed primal/dual problems and residual vectors);
 *   - optimality: zero residuals, x, z >= 0, zero gap (Section 2);
 *   - the three relative stopping inequalities on ||r_P||_2, ||r_D||_2 and the
 *     objective gap (Section 2, the three relative stopping inequalities);
 *   - the snapshot schedule of Algorithm 1 (Section 3.1): a snapshot fires when
 *     maxresid <= eps_target, then eps_target shrinks tenfold, until eps_rel.
 * Everything inside the PDHG iteration is not stated in the paper (Section 4.1
 * only says the solver closely follows cuPDLP+).  The readings used here are
 * the published PDLP-style defaults (Ruiz equilibration, power-iteration step
 * size, primal weight, averaged iterates with KKT-based adaptive restarts);
 * each one is named where it is implemented.
 *
 * Rounding: IEEE binary64, round to nearest; build with -O2 -ffp-contract=off
 * -fno-fast-math so that every operation below is rounded as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ---------------------------------------------------------------- types -- */

typedef struct {
    int64_t m, n;
    const int64_t *rp;   /* row pointers, m+1 */
    const int32_t *ci;   /* column indices, nnz */
} or_pattern;

/* Parameters (mirrored by ctypes in oracle.py; layout must match). */
typedef struct {
    int32_t ruiz_passes;        /* Ruiz l_inf passes (10) */
    int32_t power_iters;        /* power-iteration steps (100) */
    int32_t eval_every;         /* iterations between evaluations (64) */
    int32_t literal_snapshots;  /* 1: one snapshot level per evaluation */
    int32_t variant;            /* 0 averaged (PDLP-style), 1 reflected Halpern */
    int32_t pad0_;
    double eps_rel;             /* termination tolerance on maxresid */
    double eta;                 /* step size; <= 0: 0.9 / sigma_hat */
    double omega0;              /* primal weight; <= 0: ||c~|| / ||b~|| */
    double eta_factor;          /* 0.9 */
    double beta_suff, beta_nec, beta_art, omega_theta;  /* 0.2 0.8 0.36 0.5 */
    double reflect;             /* Halpern reflection rho (1) */
    int64_t max_iters;
    double time_limit_s;
    int32_t n_levels;
    int32_t pad_;
    const double *levels;       /* descending snapshot tolerances */
    int32_t omega_rule;         /* 0 smoothed (omega_theta), 1 PID */
    int32_t pad2_;
    double pid_kp, pid_ki, pid_kd;  /* PID gains (0.99, 0.01, 0) */
    int32_t stop_on;            /* stop / candidate measure: 0 maxresid,
                                   1 rel_p only, 2 rel_d only */
    int32_t polish;             /* 1: feasibility polishing */
    double polish_frac;         /* phase budget, fraction of k (0.125) */
} or_params;

typedef struct {
    double rel_p, rel_d, rel_gap, maxresid;
    double pobj, dobj, norm_rp, norm_rd, rp_inf, rd_inf;
} or_kkt_t;

typedef struct {
    int32_t status, candidate;  /* candidate: 0 current, 1 average, 2 polished */
    int64_t iters;
    int32_t restarts, n_snap;
    int32_t n_log, polish_attempts;
    double sigma_hat, eta, omega0, omega, tau, sigma;
    double t_setup, t_iter;
    or_kkt_t kkt;
    int64_t polish_iters;       /* iterations spent in polishing phases */
} or_info;

typedef struct {
    double level;
    int64_t iter;
    double maxresid;
    int32_t candidate, pad_;
} or_snap;

enum { OR_RUNNING = 0, OR_CONVERGED = 1, OR_ITER_LIMIT = 2,
       OR_TIME_LIMIT = 3, OR_NUMERICAL = 5 };

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static double *dalloc(int64_t k) {
    double *p = (double *)calloc((size_t)(k > 0 ? k : 1), sizeof(double));
    return p;
}

/* ------------------------------------------------------ plain products -- */

/* out = A x, row by row in storage order. */
static void a_times(const or_pattern *A, const double *val, const double *x,
                    double *out) {
    for (int64_t i = 0; i < A->m; ++i) {
        double s = 0.0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p)
            s += val[p] * x[A->ci[p]];
        out[i] = s;
    }
}

/* out = A^T y, by scattering each row of A (no transpose is built). */
static void at_times(const or_pattern *A, const double *val, const double *y,
                     double *out) {
    for (int64_t j = 0; j < A->n; ++j) out[j] = 0.0;
    for (int64_t i = 0; i < A->m; ++i)
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p)
            out[A->ci[p]] += val[p] * y[i];
}

static double dot(const double *a, const double *b, int64_t k) {
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(const double *a, int64_t k) { return sqrt(dot(a, a, k)); }

/* ------------------------------------------------------ Ruiz scaling ---- */

/*
 * Ruiz l_inf equilibration (the diagonal preconditioning of the
 * method; the paper itself gives no scaling rule).  Every pass takes, from the
 * current scaled matrix (D_r,i * A_ij) * D_c,j, the row maxima rho_i and the
 * column maxima kappa_j at the same time, replaces a zero maximum by 1, and
 * divides D_r,i by sqrt(rho_i) and D_c,j by sqrt(kappa_j).  The final scaled
 * values are (D_r,i * A_ij) * D_c,j.
 */
int or_ruiz(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
            const double *v, int32_t passes, double *dr, double *dc,
            double *vs) {
    double *rho = dalloc(m), *kap = dalloc(n);
    if (!rho || !kap) { free(rho); free(kap); return -5; }
    for (int64_t i = 0; i < m; ++i) dr[i] = 1.0;
    for (int64_t j = 0; j < n; ++j) dc[j] = 1.0;
    for (int32_t pass = 0; pass < passes; ++pass) {
        for (int64_t i = 0; i < m; ++i) rho[i] = 0.0;
        for (int64_t j = 0; j < n; ++j) kap[j] = 0.0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                double a = fabs((dr[i] * v[p]) * dc[ci[p]]);
                if (a > rho[i]) rho[i] = a;
                if (a > kap[ci[p]]) kap[ci[p]] = a;
            }
        for (int64_t i = 0; i < m; ++i) {
            if (rho[i] == 0.0) rho[i] = 1.0;
            dr[i] = dr[i] / sqrt(rho[i]);
        }
        for (int64_t j = 0; j < n; ++j) {
            if (kap[j] == 0.0) kap[j] = 1.0;
            dc[j] = dc[j] / sqrt(kap[j]);
        }
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            vs[p] = (dr[i] * v[p]) * dc[ci[p]];
    free(rho);
    free(kap);
    return 0;
}

/* Scaled values (D_r,i * A_ij) * D_c,j for given, fixed factors. */
static void scale_values(int64_t m, const int64_t *rp, const int32_t *ci,
                         const double *v, const double *dr, const double *dc,
                         double *vs) {
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            vs[p] = (dr[i] * v[p]) * dc[ci[p]];
}

/* ------------------------------------------------------ power iteration - */

/*
 * Estimate of the largest singular value of the scaled matrix: start from the
 * normalised all-ones vector, apply w = A^T (A v), v = w / ||w|| for `iters`
 * steps, and return sqrt(||A^T A v||).  Returns 1 for a zero matrix.
 */
double or_power(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
                const double *vs, int32_t iters) {
    or_pattern A = {m, n, rp, ci};
    double *v = dalloc(n), *u = dalloc(m), *w = dalloc(n);
    double inv = 1.0 / sqrt((double)n);
    for (int64_t j = 0; j < n; ++j) v[j] = inv;
    for (int32_t it = 0; it < iters; ++it) {
        a_times(&A, vs, v, u);
        at_times(&A, vs, u, w);
        double nw = nrm2(w, n);
        if (!(nw > 0.0)) break;
        for (int64_t j = 0; j < n; ++j) v[j] = w[j] / nw;
    }
    a_times(&A, vs, v, u);
    at_times(&A, vs, u, w);
    double s = sqrt(nrm2(w, n));
    free(v); free(u); free(w);
    return (s > 0.0 && isfinite(s)) ? s : 1.0;
}

/* ------------------------------------------------------ KKT on the LP ---- */

/*
 * Relative KKT quantities of an unscaled pair (x, y) on the original data.
 * z is taken as max(0, c - A^T y) (the paper leaves z of a PDHG iterate open;
 * this choice makes z >= 0 and r_D = A^T y + z - c = max(0, A^T y - c)).
 * Objectives: c^T x and b^T y + l^T z.  Relative errors follow the three
 * stopping inequalities of Section 2; maxresid is their maximum.
 */
static void kkt_unscaled(const or_pattern *A, const double *val,
                         const double *b, const double *c, const double *l,
                         double nb, double nc, const double *x,
                         const double *y, double *w_m, double *w_n,
                         or_kkt_t *k) {
    a_times(A, val, x, w_m);
    at_times(A, val, y, w_n);
    double srp = 0.0, rpi = 0.0, srd = 0.0, rdi = 0.0, lz = 0.0;
    for (int64_t i = 0; i < A->m; ++i) {
        double r = b[i] - w_m[i];
        srp += r * r;
        if (fabs(r) > rpi) rpi = fabs(r);
    }
    for (int64_t j = 0; j < A->n; ++j) {
        double d = c[j] - w_n[j];
        double z = d > 0.0 ? d : 0.0;
        double rd = z - d;                 /* A^T y + z - c */
        srd += rd * rd;
        if (fabs(rd) > rdi) rdi = fabs(rd);
        if (l) lz += l[j] * z;
    }
    k->pobj = dot(c, x, A->n);
    k->dobj = dot(b, y, A->m) + lz;
    k->norm_rp = sqrt(srp);
    k->norm_rd = sqrt(srd);
    k->rp_inf = rpi;
    k->rd_inf = rdi;
    k->rel_p = k->norm_rp / (1.0 + nb);
    k->rel_d = k->norm_rd / (1.0 + nc);
    k->rel_gap = fabs(k->pobj - k->dobj) /
                 (1.0 + fabs(k->pobj) + fabs(k->dobj));
    double mr = k->rel_p;
    if (k->rel_d > mr) mr = k->rel_d;
    if (k->rel_gap > mr) mr = k->rel_gap;
    k->maxresid = mr;
    if (!isfinite(k->rel_p) || !isfinite(k->rel_d) || !isfinite(k->rel_gap))
        k->maxresid = NAN;
}

/* Exported: KKT of an unscaled (x, y); z = max(0, c - A^T y) written if z. */
int or_kkt(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
           const double *v, const double *b, const double *c, const double *l,
           const double *x, const double *y, double *z, or_kkt_t *out) {
    or_pattern A = {m, n, rp, ci};
    double *wm = dalloc(m), *wn = dalloc(n);
    if (!wm || !wn) { free(wm); free(wn); return -5; }
    kkt_unscaled(&A, v, b, c, l, nrm2(b, m), nrm2(c, n), x, y, wm, wn, out);
    if (z) {
        at_times(&A, v, y, wn);
        for (int64_t j = 0; j < n; ++j) {
            double d = c[j] - wn[j];
            z[j] = d > 0.0 ? d : 0.0;
        }
    }
    free(wm); free(wn);
    return 0;
}

/* ------------------------------------------------------ snapshot levels -- */

/*
 * Algorithm 1's targets: eps_cross, eps_cross/10, ... while above eps_rel,
 * then eps_rel itself (the main thread's final tolerance).  The levels are
 * formed as eps_cross / 10^j rather than by repeated multiplication by 0.1,
 * whose rounding would put a spurious level just above eps_rel.  Returns the
 * number of levels written (at most cap).
 */
int or_alg1_levels(double eps_cross, double eps_rel, double *out, int cap) {
    int k = 0;
    for (int j = 0; j < 64 && k < cap; ++j) {
        double lev = eps_cross / pow(10.0, (double)j);
        if (lev <= eps_rel * (1.0 + 1e-9)) break;
        out[k++] = lev;
    }
    if (k < cap) out[k++] = eps_rel;
    return k;
}

/* ------------------------------------------------------ the solver ------ */

typedef struct {
    or_kkt_t kkt;          /* original-problem relative KKT */
    double sP2, sD2, sG;   /* scaled-problem pieces of KKT_omega */
    double dx2, dy2;       /* squared distance to the last restart point */
    int finite;
} cand_t;

typedef struct {
    or_pattern A;
    const double *v, *vs, *b, *c, *l, *bs, *cs, *ls, *dr, *dc;
    double nb, nc;
    double *wm, *wn, *wm2, *wn2, *xu, *yu; /* scratch */
} prob_t;

/*
 * Statistics of a scaled candidate (xs, ys): the original-problem KKT after
 * unscaling x = D_c xs, y = D_r ys, and on the scaled problem the pieces of
 *   KKT_omega = sqrt(omega^2 ||b~ - A~ xs||^2 + ||r~_D||^2 / omega^2 + gap~^2)
 * with gap~ = c~^T xs - b~^T ys - l~^T z~, z~ = max(0, c~ - A~^T ys).
 */
static void eval_cand(prob_t *P, const double *xs, const double *ys,
                      const double *xl, const double *yl, cand_t *o) {
    int64_t m = P->A.m, n = P->A.n;
    for (int64_t j = 0; j < n; ++j) P->xu[j] = P->dc[j] * xs[j];
    for (int64_t i = 0; i < m; ++i) P->yu[i] = P->dr[i] * ys[i];
    kkt_unscaled(&P->A, P->v, P->b, P->c, P->l, P->nb, P->nc, P->xu, P->yu,
                 P->wm, P->wn, &o->kkt);
    a_times(&P->A, P->vs, xs, P->wm2);
    at_times(&P->A, P->vs, ys, P->wn2);
    double sp = 0.0, sd = 0.0, lz = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double r = P->bs[i] - P->wm2[i];
        sp += r * r;
    }
    for (int64_t j = 0; j < n; ++j) {
        double d = P->cs[j] - P->wn2[j];
        double z = d > 0.0 ? d : 0.0;
        double rd = z - d;
        sd += rd * rd;
        lz += P->ls[j] * z;
    }
    o->sP2 = sp;
    o->sD2 = sd;
    o->sG = dot(P->cs, xs, n) - dot(P->bs, ys, m) - lz;
    double dx = 0.0, dy = 0.0;
    for (int64_t j = 0; j < n; ++j) dx += (xs[j] - xl[j]) * (xs[j] - xl[j]);
    for (int64_t i = 0; i < m; ++i) dy += (ys[i] - yl[i]) * (ys[i] - yl[i]);
    o->dx2 = dx;
    o->dy2 = dy;
    o->finite = isfinite(o->kkt.maxresid) && isfinite(sp) && isfinite(sd) &&
                isfinite(o->sG);
}

static double kkt_w(const cand_t *c, double w) {
    return sqrt(w * w * c->sP2 + c->sD2 / (w * w) + c->sG * c->sG);
}

static void write_unscaled(prob_t *P, const double *xs, const double *ys,
                           double *x, double *y, double *z) {
    int64_t m = P->A.m, n = P->A.n;
    for (int64_t j = 0; j < n; ++j) P->xu[j] = P->dc[j] * xs[j];
    for (int64_t i = 0; i < m; ++i) P->yu[i] = P->dr[i] * ys[i];
    if (x) memcpy(x, P->xu, (size_t)n * sizeof(double));
    if (y) memcpy(y, P->yu, (size_t)m * sizeof(double));
    if (z) {
        at_times(&P->A, P->v, P->yu, P->wn);
        for (int64_t j = 0; j < n; ++j) {
            double d = P->c[j] - P->wn[j];
            z[j] = d > 0.0 ? d : 0.0;
        }
    }
}

/*
 * Restarted averaged PDHG (PDLP-style reading; the paper states no PDHG
 * internals).  One iteration:
 *   x_{k+1} = max(l~, x_k - tau (c~ - A~^T y_k))
 *   y_{k+1} = y_k + sigma (b~ - A~ (2 x_{k+1} - x_k))
 * with uniform averages of the iterates since the last restart.  Every
 * eval_every iterations (and once at k = 0) both candidates (current and
 * average) are evaluated; Algorithm 1's snapshot test and the eps_rel stop use
 * the candidate with the smaller maxresid; then the adaptive restart rule runs
 * on KKT_omega.  Inputs x0/y0 and outputs are unscaled.
 */
/* Outer-progress test used by refinement: the inner iterate (xs, ys) of a
 * correction LP maps to the refined point x = max(0, xo + D_c xs / DP),
 * y = yo + D_r ys / DD, whose KKT on the original data (A, bo, co) is
 * compared with `target`. */
typedef struct {
    const double *xo, *yo, *bo, *co;
    double DP, DD, nbo, nco, target;
} outer_t;

static int outer_reached(const or_pattern *A, const double *v,
                         const double *dr, const double *dc,
                         const double *xs, const double *ys,
                         const outer_t *o) {
    int64_t m = A->m, n = A->n;
    double *x = dalloc(n), *y = dalloc(m), *wm = dalloc(m), *wn = dalloc(n);
    for (int64_t j = 0; j < n; ++j) {
        double t = o->xo[j] + (dc[j] * xs[j]) / o->DP;
        x[j] = t < 0.0 ? 0.0 : t;
    }
    for (int64_t i = 0; i < m; ++i) y[i] = o->yo[i] + (dr[i] * ys[i]) / o->DD;
    or_kkt_t K;
    kkt_unscaled(A, v, o->bo, o->co, NULL, o->nbo, o->nco, x, y, wm, wn, &K);
    free(x); free(y); free(wm); free(wn);
    return K.maxresid <= o->target;
}

/*
 * Primal-weight update at a restart, from the distances dx, dy that x and y
 * travelled since the previous restart (PDLP's balancing idea: omega should
 * track ||dy|| / ||dx||).  Rule 0 moves log omega the fraction theta of the
 * way to log(dy / dx).  Rule 1 (the cuPDLP+ family's controller, read here as
 * PID control of log omega) takes the error e = log(omega dx / dy) and sets
 *   log omega <- log omega - (kp e + ki sum(e) + kd (e - e_prev)).
 * Both leave omega unchanged when either distance is below 1e-10.
 */
typedef struct {
    double integral, e_prev;
} or_pid;

static double omega_update(const or_params *prm, or_pid *pid, double omega,
                           double dx, double dy) {
    if (!(dx > 1e-10 && dy > 1e-10)) return omega;
    if (prm->omega_rule == 1) {
        const double e = log(omega * dx / dy);
        pid->integral += e;
        const double lw = log(omega) - (prm->pid_kp * e +
                                        prm->pid_ki * pid->integral +
                                        prm->pid_kd * (e - pid->e_prev));
        pid->e_prev = e;
        return exp(lw);
    }
    return exp(prm->omega_theta * log(dy / dx) +
               (1.0 - prm->omega_theta) * log(omega));
}

/* The measure a solve stops on and picks its candidate by: maxresid, or
 * for a feasibility phase only the relative primal or dual residual. */
static double stop_metric(const or_params *prm, const or_kkt_t *K) {
    return prm->stop_on == 1 ? K->rel_p : prm->stop_on == 2 ? K->rel_d
                                                            : K->maxresid;
}

static int solve_impl(int64_t m, int64_t n, const int64_t *rp,
             const int32_t *ci, const double *v, const double *b,
             const double *c, const double *l, const double *x0,
             const double *y0, const or_params *prm, or_info *info,
             double *x_out, double *y_out, double *z_out, or_snap *snaps,
             double *snap_x, double *snap_y, double *snap_z, int32_t trace_k,
             double *trace_x, double *trace_y, int32_t log_cap,
             double *eval_log, const outer_t *outer);

/*
 * Feasibility polishing (the PDLP procedure the paper's closing discussion
 * describes: PDHG phases with a zero objective inside the solve).  Read
 * here as: at an evaluation at iteration k whose candidate (x, y) already
 * has a relative gap <= eps_rel but is not yet converged, and once k has
 * reached the next polishing point,
 *   1. primal phase: PDHG (same variant, same step size eta and primal
 *      weight omega, same scaling) on  min 0 s.t. Ax = b, x >= l  from (x, 0),
 *      until rel_p <= eps_rel or a budget of max(eval_every,
 *      ceil(polish_frac k / eval_every) eval_every) iterations;
 *   2. dual phase: PDHG on  min c^T x s.t. Ax = 0, x >= 0  (the dual
 *      feasibility problem: its dual asks for c - A^T y >= 0) from (0, y),
 *      until rel_d <= eps_rel or the same budget;
 *   3. if both phases succeed and the pair (x_p, y_d) has maxresid <= eps_rel
 *      on the original LP, the solve stops with it; otherwise the main
 *      iteration continues untouched and the next polishing point is 2k.
 * x, y are unscaled; on success xp (n), yd (m) hold the polished pair and K
 * its KKT.  Returns 1 on success.
 */
static int polish_attempt(int64_t m, int64_t n, const int64_t *rp,
                          const int32_t *ci, const double *v, const double *b,
                          const double *c, const double *l, const double *x,
                          const double *y, const or_params *prm, double eta,
                          double omega, int64_t k, double *xp, double *yd,
                          or_kkt_t *K, int64_t *iters) {
    const int64_t E = prm->eval_every;
    int64_t budget = (int64_t)ceil(prm->polish_frac * (double)k / (double)E) * E;
    if (budget < E) budget = E;
    or_params ph = *prm;
    ph.eta = eta;
    ph.omega0 = omega;
    ph.max_iters = budget;
    ph.n_levels = 0;
    ph.levels = NULL;
    ph.polish = 0;
    ph.literal_snapshots = 0;
    double *zero_n = dalloc(n), *zero_m = dalloc(m);   /* stay zero */
    double *sx = dalloc(n), *sy = dalloc(m), *sz = dalloc(n);  /* scratch */
    or_info ip, id;
    int ok = 0;
    ph.stop_on = 1;
    solve_impl(m, n, rp, ci, v, b, zero_n, l, x, NULL, &ph, &ip, xp, sy, sz,
               NULL, NULL, NULL, NULL, 0, NULL, NULL, 0, NULL, NULL);
    *iters += ip.iters;
    if (ip.status == OR_CONVERGED) {
        ph.stop_on = 2;
        solve_impl(m, n, rp, ci, v, zero_m, c, NULL, NULL, y, &ph, &id, sx,
                   yd, sz, NULL, NULL, NULL, NULL, 0, NULL, NULL, 0, NULL,
                   NULL);
        *iters += id.iters;
        if (id.status == OR_CONVERGED) {
            or_kkt(m, n, rp, ci, v, b, c, l, xp, yd, NULL, K);
            ok = K->maxresid <= prm->eps_rel;
        }
    }
    free(zero_n); free(zero_m); free(sx); free(sy); free(sz);
    return ok;
}

/*
 * Reflected Halpern PDHG with restarts (the variant the cuPDLP+ line of work
 * uses; the paper's solver follows it per Section 4.1 but states no details).
 * With T(z) the PDHG step of the averaged variant applied to z = (x, y),
 *   z <- lambda ((1 + rho) T(z) - rho z) + (1 - lambda) z_0,
 *   lambda = (t + 1) / (t + 2), t = steps since the last restart (0 first),
 * anchored at the restart point z_0.  The Halpern iterate z itself is not
 * projected (it may leave x >= l), so every eval_every steps (and at k = 0)
 * the candidate for Algorithm 1's test, the eps_rel stop and the returned
 * solution is T(z), which is; z's own KKT is only logged.  Restarts test the
 * fixed-point residual r(z) = sqrt(omega ||x - T_x(z)||^2 +
 * ||y - T_y(z)||^2 / omega) against the value at the last restart (reading:
 * taken as r of the iterate the restart started from, re-weighted with the
 * new omega) and the previous check, with the same thresholds as the averaged
 * variant, and restart at T(z) with the same primal-weight update.
 */
static void pdhg_step(const or_pattern *A, const double *vs, const double *bs,
                      const double *cs, const double *ls, double tau,
                      double sigma, const double *xs, const double *ys,
                      double *xh, double *yh, double *wm, double *wn,
                      double *xe) {
    int64_t m = A->m, n = A->n;
    at_times(A, vs, ys, wn);
    for (int64_t j = 0; j < n; ++j) {
        double vj = xs[j] - tau * (cs[j] - wn[j]);
        xh[j] = vj < ls[j] ? ls[j] : vj;
    }
    for (int64_t j = 0; j < n; ++j) xe[j] = 2.0 * xh[j] - xs[j];
    a_times(A, vs, xe, wm);
    for (int64_t i = 0; i < m; ++i) yh[i] = ys[i] + sigma * (bs[i] - wm[i]);
}

static int outer_reached(const or_pattern *A, const double *v,
                         const double *dr, const double *dc,
                         const double *xs, const double *ys,
                         const outer_t *o);

static int solve_halpern(int64_t m, int64_t n, const int64_t *rp,
             const int32_t *ci, const double *v, const double *b,
             const double *c, const double *l, const double *x0,
             const double *y0, const or_params *prm, or_info *info,
             double *x_out, double *y_out, double *z_out, or_snap *snaps,
             double *snap_x, double *snap_y, double *snap_z, int32_t trace_k,
             double *trace_x, double *trace_y, int32_t log_cap,
             double *eval_log, const outer_t *outer) {
    double t0 = now_s();
    or_pattern A = {m, n, rp, ci};
    int64_t nnz = rp[m];
    for (int j = 1; j < prm->n_levels; ++j)
        if (!(prm->levels[j] < prm->levels[j - 1])) return -1;
    if (prm->eval_every < 1) return -1;
    double *vs = dalloc(nnz), *dr = dalloc(m), *dc = dalloc(n);
    double *bs = dalloc(m), *cs = dalloc(n), *ls = dalloc(n);
    double *xs = dalloc(n), *ys = dalloc(m), *xh = dalloc(n), *yh = dalloc(m);
    double *xe = dalloc(n), *xa = dalloc(n), *ya = dalloc(m);  /* anchor */
    double *wm = dalloc(m), *wn = dalloc(n), *wm2 = dalloc(m),
           *wn2 = dalloc(n), *xu = dalloc(n), *yu = dalloc(m);
    double *zero_l = dalloc(n);
    double *xcu = dalloc(n), *ycu = dalloc(m), *xpb = dalloc(n), *ydb = dalloc(m);
    or_ruiz(m, n, rp, ci, v, prm->ruiz_passes, dr, dc, vs);
    const double *lv = l ? l : zero_l;
    for (int64_t i = 0; i < m; ++i) bs[i] = dr[i] * b[i];
    for (int64_t j = 0; j < n; ++j) cs[j] = dc[j] * c[j];
    for (int64_t j = 0; j < n; ++j) ls[j] = lv[j] / dc[j];
    double sigma_hat = 0.0, eta;
    if (prm->eta > 0.0) {
        eta = prm->eta;
    } else {
        sigma_hat = or_power(m, n, rp, ci, vs, prm->power_iters);
        eta = prm->eta_factor / sigma_hat;
    }
    double nbs = nrm2(bs, m), ncs = nrm2(cs, n), omega;
    if (prm->omega0 > 0.0)
        omega = prm->omega0;
    else
        omega = (nbs > 1e-10 && ncs > 1e-10) ? ncs / nbs : 1.0;
    const double omega0 = omega, rho = prm->reflect;
    double tau = eta / omega, sigma = eta * omega;
    or_pid pid = {0.0, 0.0};
    prob_t P = {A, v, vs, b, c, lv, bs, cs, ls, dr, dc, nrm2(b, m), nrm2(c, n),
                wm2, wn2, wm2, wn2, xu, yu};
    /* eval_cand uses wm/wn (first pair) as scratch too: give it its own */
    P.wm = dalloc(m);
    P.wn = dalloc(n);
    for (int64_t j = 0; j < n; ++j) xs[j] = x0 ? x0[j] / dc[j] : 0.0;
    for (int64_t i = 0; i < m; ++i) ys[i] = y0 ? y0[i] / dr[i] : 0.0;
    memcpy(xa, xs, (size_t)n * sizeof(double));
    memcpy(ya, ys, (size_t)m * sizeof(double));
    double t1 = now_s();
    int status = OR_RUNNING, restarts = 0, n_snap = 0, next_level = 0;
    int returned = 0, n_log = 0, polish_attempts = 0;
    int64_t k = 0, t = 0, next_polish = 0, polish_iters = 0;
    double r_last = INFINITY, r_prev = INFINITY;
    cand_t Sc, Sh;
    or_kkt_t final_kkt;
    memset(&final_kkt, 0, sizeof final_kkt);
    for (;;) {
        if (k % prm->eval_every == 0) {
            /* both candidates: z and T(z) */
            pdhg_step(&A, vs, bs, cs, ls, tau, sigma, xs, ys, xh, yh, wm, wn, xe);
            eval_cand(&P, xs, ys, xa, ya, &Sc);
            eval_cand(&P, xh, yh, xa, ya, &Sh);
            double fx = 0.0, fy = 0.0;
            for (int64_t j = 0; j < n; ++j) fx += (xs[j] - xh[j]) * (xs[j] - xh[j]);
            for (int64_t i = 0; i < m; ++i) fy += (ys[i] - yh[i]) * (ys[i] - yh[i]);
            const double r_cur = sqrt(omega * fx + fy / omega);
            const int bi = 1;
            const cand_t *best = &Sh;
            int restarted = 0, polish_due = 0;
            if (!Sc.finite || !Sh.finite || !isfinite(r_cur)) {
                status = OR_NUMERICAL;
            } else {
                while (next_level < prm->n_levels &&
                       best->kkt.maxresid <= prm->levels[next_level]) {
                    snaps[n_snap].level = prm->levels[next_level];
                    snaps[n_snap].iter = k;
                    snaps[n_snap].maxresid = best->kkt.maxresid;
                    snaps[n_snap].candidate = bi;
                    if (snap_x)
                        write_unscaled(&P, bi ? xh : xs, bi ? yh : ys,
                                       snap_x + (int64_t)n_snap * n,
                                       snap_y + (int64_t)n_snap * m,
                                       snap_z + (int64_t)n_snap * n);
                    ++n_snap; ++next_level;
                    if (prm->literal_snapshots) break;
                }
                if (stop_metric(prm, &best->kkt) <= prm->eps_rel) {
                    status = OR_CONVERGED;
                    returned = bi;
                    final_kkt = best->kkt;
                    if (bi) {
                        memcpy(xs, xh, (size_t)n * sizeof(double));
                        memcpy(ys, yh, (size_t)m * sizeof(double));
                    }
                } else if (k == 0) {
                    r_last = r_cur;
                } else {
                    polish_due = prm->polish && best->kkt.rel_gap <= prm->eps_rel &&
                                 k >= next_polish;
                    if (polish_due) write_unscaled(&P, xh, yh, xcu, ycu, NULL);
                    const int r = (r_cur <= prm->beta_suff * r_last) ||
                                  (r_cur <= prm->beta_nec * r_last && r_cur > r_prev) ||
                                  ((double)t >= prm->beta_art * (double)k);
                    if (r) {
                        omega = omega_update(prm, &pid, omega, sqrt(Sh.dx2),
                                             sqrt(Sh.dy2));
                        tau = eta / omega;
                        sigma = eta * omega;
                        memcpy(xs, xh, (size_t)n * sizeof(double));
                        memcpy(ys, yh, (size_t)m * sizeof(double));
                        memcpy(xa, xh, (size_t)n * sizeof(double));
                        memcpy(ya, yh, (size_t)m * sizeof(double));
                        t = 0;
                        r_last = sqrt(omega * fx + fy / omega);
                        r_prev = INFINITY;
                        ++restarts;
                        restarted = 1;
                    } else {
                        r_prev = r_cur;
                    }
                }
            }
            if (polish_due) {
                or_kkt_t pk;
                ++polish_attempts;
                if (polish_attempt(m, n, rp, ci, v, b, c, l, xcu, ycu, prm, eta,
                                   omega, k, xpb, ydb, &pk, &polish_iters)) {
                    status = OR_CONVERGED;
                    returned = 2;
                    final_kkt = pk;
                    for (int64_t j = 0; j < n; ++j) xs[j] = xpb[j] / dc[j];
                    for (int64_t i = 0; i < m; ++i) ys[i] = ydb[i] / dr[i];
                } else {
                    next_polish = 2 * k;
                }
            }
            if (eval_log && n_log < log_cap) {
                double *e = eval_log + 8 * (int64_t)n_log++;
                e[0] = (double)k; e[1] = Sc.kkt.maxresid; e[2] = Sh.kkt.maxresid;
                e[3] = r_cur; e[4] = r_last; e[5] = (double)restarted;
                e[6] = 1.0; e[7] = omega;
            }
            if (status == OR_RUNNING && outer && !restarted &&
                outer_reached(&A, v, dr, dc, xh, yh, outer)) {
                status = OR_CONVERGED;
                returned = 1;
                final_kkt = Sh.kkt;
                memcpy(xs, xh, (size_t)n * sizeof(double));
                memcpy(ys, yh, (size_t)m * sizeof(double));
            } else if (status == OR_RUNNING && outer && restarted &&
                       outer_reached(&A, v, dr, dc, xs, ys, outer)) {
                /* after a restart the current iterate already is T(z) */
                status = OR_CONVERGED;
                returned = 1;
                final_kkt = Sh.kkt;
            }
            if (status == OR_RUNNING && prm->time_limit_s > 0.0 &&
                now_s() - t0 > prm->time_limit_s)
                status = OR_TIME_LIMIT;
        }
        /* trace: the iterate after step k and the evaluation due at k */
        if (k >= 1 && k <= trace_k && trace_x) {
            for (int64_t j = 0; j < n; ++j) trace_x[(k - 1) * n + j] = dc[j] * xs[j];
            for (int64_t i = 0; i < m; ++i) trace_y[(k - 1) * m + i] = dr[i] * ys[i];
        }
        if (status != OR_RUNNING) break;
        if (k >= prm->max_iters) { status = OR_ITER_LIMIT; break; }
        /* one reflected Halpern step */
        pdhg_step(&A, vs, bs, cs, ls, tau, sigma, xs, ys, xh, yh, wm, wn, xe);
        const double lam = (double)(t + 1) / (double)(t + 2);
        for (int64_t j = 0; j < n; ++j)
            xs[j] = lam * ((1.0 + rho) * xh[j] - rho * xs[j]) + (1.0 - lam) * xa[j];
        for (int64_t i = 0; i < m; ++i)
            ys[i] = lam * ((1.0 + rho) * yh[i] - rho * ys[i]) + (1.0 - lam) * ya[i];
        ++k; ++t;
    }
    double t2 = now_s();
    if (status != OR_CONVERGED) {
        cand_t S;
        eval_cand(&P, xs, ys, xa, ya, &S);
        final_kkt = S.kkt;
        returned = 0;
    }
    write_unscaled(&P, xs, ys, x_out, y_out, z_out);
    if (info) {
        info->status = status;
        info->candidate = returned;
        info->iters = k;
        info->restarts = restarts;
        info->n_snap = n_snap;
        info->n_log = n_log;
        info->polish_attempts = polish_attempts;
        info->polish_iters = polish_iters;
        info->sigma_hat = sigma_hat;
        info->eta = eta;
        info->omega0 = omega0;
        info->omega = omega;
        info->tau = tau;
        info->sigma = sigma;
        info->t_setup = t1 - t0;
        info->t_iter = t2 - t1;
        info->kkt = final_kkt;
    }
    free(vs); free(dr); free(dc); free(bs); free(cs); free(ls); free(xs);
    free(ys); free(xh); free(yh); free(xe); free(xa); free(ya); free(wm);
    free(wn); free(wm2); free(wn2); free(xu); free(yu); free(zero_l);
    free(P.wm); free(P.wn);
    free(xcu); free(ycu); free(xpb); free(ydb);
    return 0;
}

static int solve_impl(int64_t m, int64_t n, const int64_t *rp,
             const int32_t *ci, const double *v, const double *b,
             const double *c, const double *l, const double *x0,
             const double *y0, const or_params *prm, or_info *info,
             double *x_out, double *y_out, double *z_out, or_snap *snaps,
             double *snap_x, double *snap_y, double *snap_z, int32_t trace_k,
             double *trace_x, double *trace_y, int32_t log_cap,
             double *eval_log, const outer_t *outer) {
    if (prm->variant == 1)
        return solve_halpern(m, n, rp, ci, v, b, c, l, x0, y0, prm, info,
                             x_out, y_out, z_out, snaps, snap_x, snap_y,
                             snap_z, trace_k, trace_x, trace_y, log_cap,
                             eval_log, outer);
    double t0 = now_s();
    or_pattern A = {m, n, rp, ci};
    int64_t nnz = rp[m];
    for (int j = 1; j < prm->n_levels; ++j)
        if (!(prm->levels[j] < prm->levels[j - 1])) return -1;
    if (prm->eval_every < 1) return -1;

    double *vs = dalloc(nnz), *dr = dalloc(m), *dc = dalloc(n);
    double *bs = dalloc(m), *cs = dalloc(n), *ls = dalloc(n);
    double *xs = dalloc(n), *ys = dalloc(m), *xn = dalloc(n), *xe = dalloc(n);
    double *xbar = dalloc(n), *ybar = dalloc(m), *xl = dalloc(n),
           *yl = dalloc(m);
    double *wm = dalloc(m), *wn = dalloc(n), *wm2 = dalloc(m),
           *wn2 = dalloc(n), *xu = dalloc(n), *yu = dalloc(m);
    double *zero_l = dalloc(n);
    /* polishing: the candidate (unscaled) and the polished pair */
    double *xcu = dalloc(n), *ycu = dalloc(m), *xpb = dalloc(n), *ydb = dalloc(m);

    or_ruiz(m, n, rp, ci, v, prm->ruiz_passes, dr, dc, vs);
    const double *lv = l ? l : zero_l;
    for (int64_t i = 0; i < m; ++i) bs[i] = dr[i] * b[i];
    for (int64_t j = 0; j < n; ++j) cs[j] = dc[j] * c[j];
    for (int64_t j = 0; j < n; ++j) ls[j] = lv[j] / dc[j];

    double sigma_hat = 0.0, eta;
    if (prm->eta > 0.0) {
        eta = prm->eta;
    } else {
        sigma_hat = or_power(m, n, rp, ci, vs, prm->power_iters);
        eta = prm->eta_factor / sigma_hat;
    }
    double nbs = nrm2(bs, m), ncs = nrm2(cs, n), omega;
    if (prm->omega0 > 0.0)
        omega = prm->omega0;
    else
        omega = (nbs > 1e-10 && ncs > 1e-10) ? ncs / nbs : 1.0;
    double omega0 = omega;
    double tau = eta / omega, sigma = eta * omega;
    or_pid pid = {0.0, 0.0};

    prob_t P = {A, v, vs, b, c, lv, bs, cs, ls, dr, dc, nrm2(b, m), nrm2(c, n),
                wm, wn, wm2, wn2, xu, yu};

    for (int64_t j = 0; j < n; ++j) xs[j] = x0 ? x0[j] / dc[j] : 0.0;
    for (int64_t i = 0; i < m; ++i) ys[i] = y0 ? y0[i] / dr[i] : 0.0;
    memcpy(xl, xs, (size_t)n * sizeof(double));
    memcpy(yl, ys, (size_t)m * sizeof(double));
    double t1 = now_s();

    int status = OR_RUNNING, restarts = 0, n_snap = 0, next_level = 0;
    int returned = 0, n_log = 0, polish_attempts = 0;
    int64_t k = 0, t = 0, next_polish = 0, polish_iters = 0;
    double K_last, K_prev = INFINITY;
    cand_t Sc, Sa, *best;
    or_kkt_t final_kkt;

    /* evaluation at k = 0: current iterate only, no restart */
    eval_cand(&P, xs, ys, xl, yl, &Sc);
    K_last = kkt_w(&Sc, omega);
    if (!Sc.finite) status = OR_NUMERICAL;
    while (status == OR_RUNNING && next_level < prm->n_levels &&
           Sc.kkt.maxresid <= prm->levels[next_level]) {
        snaps[n_snap].level = prm->levels[next_level];
        snaps[n_snap].iter = 0;
        snaps[n_snap].maxresid = Sc.kkt.maxresid;
        snaps[n_snap].candidate = 0;
        if (snap_x)
            write_unscaled(&P, xs, ys, snap_x + (int64_t)n_snap * n,
                           snap_y + (int64_t)n_snap * m,
                           snap_z + (int64_t)n_snap * n);
        ++n_snap; ++next_level;
        if (prm->literal_snapshots) break;
    }
    if (status == OR_RUNNING && stop_metric(prm, &Sc.kkt) <= prm->eps_rel)
        status = OR_CONVERGED;
    final_kkt = Sc.kkt;
    if (eval_log && n_log < log_cap) {
        double *e = eval_log + 8 * (int64_t)n_log++;
        e[0] = 0.0; e[1] = Sc.kkt.maxresid; e[2] = NAN; e[3] = K_last;
        e[4] = INFINITY; e[5] = 0.0; e[6] = 0.0; e[7] = omega;
    }

    while (status == OR_RUNNING) {
        if (k >= prm->max_iters) { status = OR_ITER_LIMIT; break; }
        /* primal step with projection onto x >= l~ */
        at_times(&A, vs, ys, wn);
        for (int64_t j = 0; j < n; ++j) {
            double vj = xs[j] - tau * (cs[j] - wn[j]);
            xn[j] = vj < ls[j] ? ls[j] : vj;
        }
        /* extrapolated dual step, 2 x_{k+1} - x_k formed literally */
        for (int64_t j = 0; j < n; ++j) xe[j] = 2.0 * xn[j] - xs[j];
        a_times(&A, vs, xe, wm);
        for (int64_t i = 0; i < m; ++i) ys[i] = ys[i] + sigma * (bs[i] - wm[i]);
        memcpy(xs, xn, (size_t)n * sizeof(double));
        ++k; ++t;
        /* uniform average of the iterates since the last restart */
        for (int64_t j = 0; j < n; ++j) xbar[j] = xbar[j] + (xs[j] - xbar[j]) / (double)t;
        for (int64_t i = 0; i < m; ++i) ybar[i] = ybar[i] + (ys[i] - ybar[i]) / (double)t;

        if (k % prm->eval_every == 0) {
            eval_cand(&P, xs, ys, xl, yl, &Sc);
            eval_cand(&P, xbar, ybar, xl, yl, &Sa);
            int bi = (stop_metric(prm, &Sa.kkt) < stop_metric(prm, &Sc.kkt)) ? 1 : 0;
            best = bi ? &Sa : &Sc;
            int polish_due = 0;
            double Kc_cur = kkt_w(&Sc, omega), Kc_avg = kkt_w(&Sa, omega);
            int restarted = 0, cand = (Kc_avg < Kc_cur) ? 1 : 0;
            if (!Sc.finite || !Sa.finite) {
                status = OR_NUMERICAL;
            } else {
                /* Algorithm 1's snapshot test on the better candidate */
                while (next_level < prm->n_levels &&
                       best->kkt.maxresid <= prm->levels[next_level]) {
                    snaps[n_snap].level = prm->levels[next_level];
                    snaps[n_snap].iter = k;
                    snaps[n_snap].maxresid = best->kkt.maxresid;
                    snaps[n_snap].candidate = bi;
                    if (snap_x)
                        write_unscaled(&P, bi ? xbar : xs, bi ? ybar : ys,
                                       snap_x + (int64_t)n_snap * n,
                                       snap_y + (int64_t)n_snap * m,
                                       snap_z + (int64_t)n_snap * n);
                    ++n_snap; ++next_level;
                    if (prm->literal_snapshots) break;
                }
                if (stop_metric(prm, &best->kkt) <= prm->eps_rel) {
                    status = OR_CONVERGED;
                    returned = bi;
                    final_kkt = best->kkt;
                    if (bi) {
                        memcpy(xs, xbar, (size_t)n * sizeof(double));
                        memcpy(ys, ybar, (size_t)m * sizeof(double));
                    }
                } else {
                    /* polishing is decided on the candidate before the
                       restart test may replace it, and runs after it */
                    polish_due = prm->polish && best->kkt.rel_gap <= prm->eps_rel &&
                                 k >= next_polish;
                    if (polish_due)
                        write_unscaled(&P, bi ? xbar : xs, bi ? ybar : ys, xcu,
                                       ycu, NULL);
                    /* adaptive restart on KKT_omega */
                    const cand_t *S = cand ? &Sa : &Sc;
                    double Kc = cand ? Kc_avg : Kc_cur;
                    int r = (Kc <= prm->beta_suff * K_last) ||
                            (Kc <= prm->beta_nec * K_last && Kc > K_prev) ||
                            ((double)t >= prm->beta_art * (double)k);
                    if (r) {
                        omega = omega_update(prm, &pid, omega, sqrt(S->dx2),
                                             sqrt(S->dy2));
                        tau = eta / omega;
                        sigma = eta * omega;
                        if (cand) {
                            memcpy(xs, xbar, (size_t)n * sizeof(double));
                            memcpy(ys, ybar, (size_t)m * sizeof(double));
                        }
                        memcpy(xl, xs, (size_t)n * sizeof(double));
                        memcpy(yl, ys, (size_t)m * sizeof(double));
                        /* averages start afresh: the first one after the
                           restart is exactly the first new iterate */
                        memset(xbar, 0, (size_t)n * sizeof(double));
                        memset(ybar, 0, (size_t)m * sizeof(double));
                        t = 0;
                        K_last = kkt_w(S, omega);
                        K_prev = INFINITY;
                        ++restarts;
                        restarted = 1;
                    } else {
                        K_prev = Kc;
                    }
                }
            }
            if (polish_due) {
                or_kkt_t pk;
                ++polish_attempts;
                if (polish_attempt(m, n, rp, ci, v, b, c, l, xcu, ycu, prm, eta,
                                   omega, k, xpb, ydb, &pk, &polish_iters)) {
                    status = OR_CONVERGED;
                    returned = 2;
                    final_kkt = pk;
                    for (int64_t j = 0; j < n; ++j) xs[j] = xpb[j] / dc[j];
                    for (int64_t i = 0; i < m; ++i) ys[i] = ydb[i] / dr[i];
                } else {
                    next_polish = 2 * k;
                }
            }
            if (eval_log && n_log < log_cap) {
                double *e = eval_log + 8 * (int64_t)n_log++;
                e[0] = (double)k; e[1] = Sc.kkt.maxresid; e[2] = Sa.kkt.maxresid;
                e[3] = Kc_cur; e[4] = Kc_avg; e[5] = (double)restarted;
                e[6] = (double)cand; e[7] = omega;
            }
            /* refinement: stop as soon as the refined point has made the
               required progress on the original problem */
            if (status == OR_RUNNING && outer &&
                outer_reached(&A, v, dr, dc, xs, ys, outer)) {
                status = OR_CONVERGED;
                returned = 0;
            }
            if (status == OR_RUNNING && prm->time_limit_s > 0.0 &&
                now_s() - t0 > prm->time_limit_s)
                status = OR_TIME_LIMIT;
        }
        if (k <= trace_k && trace_x) {
            for (int64_t j = 0; j < n; ++j) trace_x[(k - 1) * n + j] = dc[j] * xs[j];
            for (int64_t i = 0; i < m; ++i) trace_y[(k - 1) * m + i] = dr[i] * ys[i];
        }
    }
    double t2 = now_s();

    if (status != OR_CONVERGED || (outer && returned == 0)) {
        cand_t S;
        eval_cand(&P, xs, ys, xl, yl, &S);
        final_kkt = S.kkt;
        returned = 0;
    }
    write_unscaled(&P, xs, ys, x_out, y_out, z_out);

    if (info) {
        info->status = status;
        info->candidate = returned;
        info->iters = k;
        info->restarts = restarts;
        info->n_snap = n_snap;
        info->n_log = n_log;
        info->polish_attempts = polish_attempts;
        info->polish_iters = polish_iters;
        info->sigma_hat = sigma_hat;
        info->eta = eta;
        info->omega0 = omega0;
        info->omega = omega;
        info->tau = tau;
        info->sigma = sigma;
        info->t_setup = t1 - t0;
        info->t_iter = t2 - t1;
        info->kkt = final_kkt;
    }
    free(vs); free(dr); free(dc); free(bs); free(cs); free(ls);
    free(xs); free(ys); free(xn); free(xe); free(xbar); free(ybar);
    free(xl); free(yl); free(wm); free(wn); free(wm2); free(wn2);
    free(xu); free(yu); free(zero_l);
    free(xcu); free(ycu); free(xpb); free(ydb);
    return 0;
}

int or_solve(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
             const double *v, const double *b, const double *c,
             const double *l, const double *x0, const double *y0,
             const or_params *prm, or_info *info, double *x_out,
             double *y_out, double *z_out, or_snap *snaps, double *snap_x,
             double *snap_y, double *snap_z, int32_t trace_k,
             double *trace_x, double *trace_y, int32_t log_cap,
             double *eval_log) {
    return solve_impl(m, n, rp, ci, v, b, c, l, x0, y0, prm, info, x_out,
                      y_out, z_out, snaps, snap_x, snap_y, snap_z, trace_k,
                      trace_x, trace_y, log_cap, eval_log, NULL);
}

/* ------------------------------------------------------ refinement ----- */

/*
 * Iterative refinement for LP (Gleixner, Steffy and Wolter's method, here
 * with PDHG inner solves; not part of the paper).  Round 0 solves the LP
 * itself.  Round r >= 1 measures, in FP64,
 *   delta_P = max(||b - Ax||_inf, max_j (-x_j)^+),  delta_D = max_j (-(c - A^T y)_j)^+
 * takes the power-of-two scale Delta = min(2^floor(log2(1/delta)), 2^cap * Delta_prev)
 * (the capped value when delta = 0), solves the correction LP
 *   min (Delta_D d)^T xh  s.t.  A xh = Delta_P r_P,  xh >= -Delta_P x
 * and updates x <- max(0, x + xh / Delta_P), y <- y + yh / Delta_D.
 * The inner solver is the PDHG above (FP64 here) with the inner parameters,
 * and two choices made for PDHG inner solves:
 *  - the inner solve also stops once the refined point reaches
 *    max(outer_eps, progress * maxresid before the round) on the original
 *    LP (checked at every inner evaluation), since the correction LP's own
 *    relative criteria are diluted by the large scaled reduced costs of
 *    nonbasic columns;
 *  - a round r >= 1 starts from the previous inner solve's final primal
 *    weight times (Delta_D / Delta_D,prev) / (Delta_P / Delta_P,prev): the
 *    correction's dual and primal solutions scale by Delta_D and Delta_P,
 *    while ||c^|| / ||b^|| is dominated by those reduced costs.
 */
int or_refine(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
              const double *v, const double *b, const double *c,
              const or_params *inner, double outer_eps, double progress,
              int32_t max_rounds, int32_t cap_log2, double *x, double *y,
              or_kkt_t *final_kkt, int32_t *rounds_done, int64_t *inner_iters,
              double *round_log) {
    or_pattern A = {m, n, rp, ci};
    double *rpv = dalloc(m), *d = dalloc(n), *bh = dalloc(m), *ch = dalloc(n),
           *lh = dalloc(n), *xh = dalloc(n), *yh = dalloc(m), *zh = dalloc(n),
           *wm = dalloc(m), *wn = dalloc(n);
    double nb = nrm2(b, m), nc = nrm2(c, n);
    double DP = 1.0, DD = 1.0, DPprev = 1.0, DDprev = 1.0, omega_end = 0.0;
    int64_t total = 0;
    int r = 0, status = OR_ITER_LIMIT;
    for (int64_t j = 0; j < n; ++j) x[j] = 0.0;
    for (int64_t i = 0; i < m; ++i) y[i] = 0.0;
    for (r = 0;; ++r) {
        or_kkt_t K;
        kkt_unscaled(&A, v, b, c, NULL, nb, nc, x, y, wm, wn, &K);
        if (round_log) {
            round_log[4 * r + 0] = K.maxresid;
            round_log[4 * r + 1] = DP;
            round_log[4 * r + 2] = DD;
            round_log[4 * r + 3] = (double)total;
        }
        *final_kkt = K;
        if (K.maxresid <= outer_eps) { status = OR_CONVERGED; break; }
        if (r >= max_rounds) break;
        a_times(&A, v, x, rpv);
        for (int64_t i = 0; i < m; ++i) rpv[i] = b[i] - rpv[i];
        at_times(&A, v, y, d);
        for (int64_t j = 0; j < n; ++j) d[j] = c[j] - d[j];
        if (r >= 1) {
            double dP = 0.0, dD = 0.0;
            for (int64_t i = 0; i < m; ++i) if (fabs(rpv[i]) > dP) dP = fabs(rpv[i]);
            for (int64_t j = 0; j < n; ++j) if (-x[j] > dP) dP = -x[j];
            for (int64_t j = 0; j < n; ++j) if (-d[j] > dD) dD = -d[j];
            DPprev = DP;
            DDprev = DD;
            double capP = ldexp(DP, cap_log2), capD = ldexp(DD, cap_log2);
            double sP = dP > 0.0 ? ldexp(1.0, (int)floor(log2(1.0 / dP))) : capP;
            double sD = dD > 0.0 ? ldexp(1.0, (int)floor(log2(1.0 / dD))) : capD;
            DP = sP < capP ? sP : capP;
            DD = sD < capD ? sD : capD;
        }
        for (int64_t i = 0; i < m; ++i) bh[i] = DP * rpv[i];
        for (int64_t j = 0; j < n; ++j) ch[j] = DD * d[j];
        for (int64_t j = 0; j < n; ++j) lh[j] = -DP * x[j];
        or_info info;
        or_snap dummy;
        or_params ip = *inner;
        ip.n_levels = 0;
        if (r >= 1 && omega_end > 0.0)
            ip.omega0 = omega_end * (DD / DDprev) / (DP / DPprev);
        outer_t oc = {x, y, b, c, DP, DD, nb, nc,
                      fmax(outer_eps, progress * K.maxresid)};
        int rc = solve_impl(m, n, rp, ci, v, bh, ch, lh, NULL, NULL, &ip,
                            &info, xh, yh, zh, &dummy, NULL, NULL, NULL, 0,
                            NULL, NULL, 0, NULL, &oc);
        omega_end = info.omega;
        if (rc != 0) { status = rc; break; }
        total += info.iters;
        for (int64_t j = 0; j < n; ++j) {
            double xv = x[j] + xh[j] / DP;
            x[j] = xv < 0.0 ? 0.0 : xv;
        }
        for (int64_t i = 0; i < m; ++i) y[i] = y[i] + yh[i] / DD;
    }
    *rounds_done = r;
    *inner_iters = total;
    free(rpv); free(d); free(bh); free(ch); free(lh); free(xh); free(yh);
    free(zh); free(wm); free(wn);
    return status;
}

/* ------------------------------------------------------ unrolled adjoint - */

/*
 * K plain PDHG steps (no restarts, no averaging) on the problem scaled by
 * the given, fixed diagonal factors D_r, D_c (in practice the Ruiz factors of
 * the unperturbed A), from (x0, y0) (unscaled; NULL: zero):
 *   x_{k+1} = max(0, v_k),  v_k = x_k - tau (c~ - A~^T y_k)
 *   y_{k+1} = y_k + sigma (b~ - A~ (2 x_{k+1} - x_k))
 * Loss L = || D_c x_K - x_t ||^2.  All K+1 iterates are stored, then the
 * reverse pass walks the steps backwards (the subgradient of the projection
 * is taken as 1[v_k > 0], i.e. 0 at a tie).  Gradients are returned for the
 * unscaled c, b and the values of A (A's CSR order), chaining through the
 * fixed scaling: dL/dc = D_c dL/dc~, dL/db = D_r dL/db~,
 * dL/dA_ij = D_r,i D_c,j dL/dA~_ij.
 */
int or_unrolled(int64_t m, int64_t n, const int64_t *rp, const int32_t *ci,
                const double *v, const double *b, const double *c,
                const double *dr, const double *dc, double tau, double sigma,
                int32_t K, const double *x0, const double *y0, const double *xt,
                double *xK, double *loss, double *gc, double *gb,
                double *gA) {
    or_pattern A = {m, n, rp, ci};
    int64_t nnz = rp[m];
    double *vs = dalloc(nnz);
    double *bs = dalloc(m), *cs = dalloc(n);
    double *X = dalloc((int64_t)(K + 1) * n), *Y = dalloc((int64_t)(K + 1) * m);
    double *wm = dalloc(m), *wn = dalloc(n), *xe = dalloc(n);
    double *gx = dalloc(n), *gy = dalloc(m), *gxk = dalloc(n), *gyk = dalloc(m);
    double *gxbar = dalloc(n), *gv = dalloc(n), *gcs = dalloc(n),
           *gbs = dalloc(m), *gAs = dalloc(nnz);
    if (!X || !Y || !gAs) return -5;

    scale_values(m, rp, ci, v, dr, dc, vs);
    for (int64_t i = 0; i < m; ++i) bs[i] = dr[i] * b[i];
    for (int64_t j = 0; j < n; ++j) cs[j] = dc[j] * c[j];
    for (int64_t j = 0; j < n; ++j) X[j] = x0 ? x0[j] / dc[j] : 0.0;
    for (int64_t i = 0; i < m; ++i) Y[i] = y0 ? y0[i] / dr[i] : 0.0;

    for (int32_t k = 0; k < K; ++k) {
        const double *xk = X + (int64_t)k * n, *yk = Y + (int64_t)k * m;
        double *xk1 = X + (int64_t)(k + 1) * n, *yk1 = Y + (int64_t)(k + 1) * m;
        at_times(&A, vs, yk, wn);
        for (int64_t j = 0; j < n; ++j) {
            double vj = xk[j] - tau * (cs[j] - wn[j]);
            xk1[j] = vj < 0.0 ? 0.0 : vj;
        }
        for (int64_t j = 0; j < n; ++j) xe[j] = 2.0 * xk1[j] - xk[j];
        a_times(&A, vs, xe, wm);
        for (int64_t i = 0; i < m; ++i) yk1[i] = yk[i] + sigma * (bs[i] - wm[i]);
    }
    const double *xKs = X + (int64_t)K * n;
    double L = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double e = dc[j] * xKs[j] - xt[j];
        xK[j] = dc[j] * xKs[j];
        L += e * e;
        gx[j] = dc[j] * (2.0 * e);          /* dL/dx~_K */
    }
    *loss = L;
    for (int64_t i = 0; i < m; ++i) gy[i] = 0.0;

    for (int32_t k = K - 1; k >= 0; --k) {
        const double *xk = X + (int64_t)k * n, *yk = Y + (int64_t)k * m;
        const double *xk1 = X + (int64_t)(k + 1) * n;
        /* gx holds dL/dx_{k+1} from later steps, gy holds dL/dy_{k+1} */
        /* dual step y_{k+1} = y_k + sigma (b~ - A~ xbar_k), xbar_k = 2x_{k+1} - x_k */
        at_times(&A, vs, gy, wn);
        for (int64_t j = 0; j < n; ++j) gxbar[j] = -sigma * wn[j];
        for (int64_t i = 0; i < m; ++i) gbs[i] += sigma * gy[i];
        for (int64_t i = 0; i < m; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                int32_t j = ci[p];
                gAs[p] += -sigma * gy[i] * (2.0 * xk1[j] - xk[j]);
            }
        for (int64_t j = 0; j < n; ++j) gx[j] += 2.0 * gxbar[j];
        for (int64_t j = 0; j < n; ++j) gxk[j] = -gxbar[j];
        for (int64_t i = 0; i < m; ++i) gyk[i] = gy[i];
        /* primal step x_{k+1} = max(0, v_k) */
        at_times(&A, vs, yk, wn);
        for (int64_t j = 0; j < n; ++j) {
            double vj = xk[j] - tau * (cs[j] - wn[j]);
            gv[j] = vj > 0.0 ? gx[j] : 0.0;
        }
        for (int64_t j = 0; j < n; ++j) gxk[j] += gv[j];
        for (int64_t j = 0; j < n; ++j) gcs[j] += -tau * gv[j];
        a_times(&A, vs, gv, wm);
        for (int64_t i = 0; i < m; ++i) gyk[i] += tau * wm[i];
        for (int64_t i = 0; i < m; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                gAs[p] += tau * yk[i] * gv[ci[p]];
        memcpy(gx, gxk, (size_t)n * sizeof(double));
        memcpy(gy, gyk, (size_t)m * sizeof(double));
    }
    for (int64_t j = 0; j < n; ++j) gc[j] = dc[j] * gcs[j];
    for (int64_t i = 0; i < m; ++i) gb[i] = dr[i] * gbs[i];
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            gA[p] = (dr[i] * gAs[p]) * dc[ci[p]];

    free(vs); free(bs); free(cs); free(X); free(Y);
    free(wm); free(wn); free(xe); free(gx); free(gy); free(gxk); free(gyk);
    free(gxbar); free(gv); free(gcs); free(gbs); free(gAs);
    return 0;
}

/* Plain forward of the same K steps (no storage), for finite differences. */
int or_unrolled_fwd(int64_t m, int64_t n, const int64_t *rp,
                    const int32_t *ci, const double *v, const double *b,
                    const double *c, const double *dr, const double *dc,
                    double tau, double sigma, int32_t K, double *xK,
                    uint64_t *mask_hash) {
    or_pattern A = {m, n, rp, ci};
    int64_t nnz = rp[m];
    double *vs = dalloc(nnz);
    double *bs = dalloc(m), *cs = dalloc(n), *x = dalloc(n), *y = dalloc(m);
    double *xn = dalloc(n), *xe = dalloc(n), *wm = dalloc(m), *wn = dalloc(n);
    uint64_t h = 1469598103934665603ull;   /* FNV-1a over the mask bits */
    scale_values(m, rp, ci, v, dr, dc, vs);
    for (int64_t i = 0; i < m; ++i) bs[i] = dr[i] * b[i];
    for (int64_t j = 0; j < n; ++j) cs[j] = dc[j] * c[j];
    for (int32_t k = 0; k < K; ++k) {
        at_times(&A, vs, y, wn);
        for (int64_t j = 0; j < n; ++j) {
            double vj = x[j] - tau * (cs[j] - wn[j]);
            xn[j] = vj < 0.0 ? 0.0 : vj;
            h = (h ^ (uint64_t)(vj > 0.0)) * 1099511628211ull;
        }
        for (int64_t j = 0; j < n; ++j) xe[j] = 2.0 * xn[j] - x[j];
        a_times(&A, vs, xe, wm);
        for (int64_t i = 0; i < m; ++i) y[i] = y[i] + sigma * (bs[i] - wm[i]);
        memcpy(x, xn, (size_t)n * sizeof(double));
    }
    for (int64_t j = 0; j < n; ++j) xK[j] = dc[j] * x[j];
    if (mask_hash) *mask_hash = h;
    free(vs); free(bs); free(cs); free(x); free(y);
    free(xn); free(xe); free(wm); free(wn);
    return 0;
}
