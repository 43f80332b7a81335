// cpu_pdhg.cpp -- the restarted PDHG on the host's cores: the paper's CPU
// platform (Section 4.1 runs its PDHG on CPU cores as well as on the GPU;
// Section 5 notes that a few cores saturate the CPU's memory bandwidth).
//
// The same method as the GPU path, in FP64: Ruiz equilibration, the power
// iteration for the step size, the averaged (PDLP-style restarts) or the
// reflected Halpern iteration, an FP64 KKT evaluation every eval_every
// iterations whose decisions (Algorithm 1's snapshot test, the eps_rel stop,
// the adaptive restart and the primal-weight update) are control_decide's,
// shared with the GPU control kernel.  Work is split over a fixed pool of
// host threads: the primal half over row ranges of A^T and the dual half over
// row ranges of A, each range holding an equal share of the nonzeros.  Every
// reduction is summed over fixed chunks of rows in chunk order, so the
// results do not depend on the thread count.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "control.h"
#include "internal.h"

using namespace pdhg;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Persistent worker threads: run(f) calls f(t) for t = 0 .. size - 1, t = 0
// on the calling thread, and returns when every call has returned.
class Pool {
  public:
    explicit Pool(int threads) : T_(threads) {
        for (int t = 1; t < T_; ++t) workers_.emplace_back([this, t] { loop(t); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            ++gen_;
        }
        cv_.notify_all();
        for (auto &w : workers_) w.join();
    }
    int size() const { return T_; }
    void run(const std::function<void(int)> &f) {
        if (T_ == 1) {
            f(0);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &f;
            done_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        f(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this] { return done_ == T_ - 1; });
        job_ = nullptr;
    }

  private:
    void loop(int t) {
        long seen = 0;
        for (;;) {
            const std::function<void(int)> *f;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
                f = job_;
            }
            (*f)(t);
            {
                std::lock_guard<std::mutex> lk(mu_);
                ++done_;
            }
            done_cv_.notify_one();
        }
    }
    int T_;
    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *job_ = nullptr;
    long gen_ = 0;
    int done_ = 0;
    bool stop_ = false;
};

// Row ranges of equal nonzero count (each row also counts one, so runs of
// empty rows are shared out too).
std::vector<int64_t> split_rows(int64_t rows, const int64_t *rp, int parts) {
    std::vector<int64_t> cut((size_t)parts + 1, rows);
    cut[0] = 0;
    const double total = (double)rp[rows] + (double)rows;
    int64_t r = 0;
    for (int p = 1; p < parts; ++p) {
        const double goal = total * p / parts;
        while (r < rows && (double)rp[r] + (double)r < goal) ++r;
        cut[p] = r;
    }
    return cut;
}

constexpr int64_t kChunk = 4096;   // rows per reduction chunk

struct SnapCopy {
    pdhg_snapshot_info info;
    std::vector<double> x, y, z;
};

}  // namespace

struct pdhg_cpu {
    std::unique_ptr<Pool> pool;
    std::string err;
    bool loaded = false, configured = false;
    int64_t m = 0, n = 0, nnz = 0;
    std::vector<int64_t> arp, atrp, perm;
    std::vector<int32_t> aci, atci;
    std::vector<double> av, atv;          // loaded values
    std::vector<double> as, ats;          // scaled values
    std::vector<double> b0, c0, l0;
    bool has_l = false;
    std::vector<double> dr, dc, bs, cs, ls;
    std::vector<int64_t> cut_a, cut_at;   // thread row ranges of A, A^T
    // iterate (scaled): current, average (Halpern: T(z)), restart point,
    // A~ x of the current iterate and of the Halpern anchor
    std::vector<double> x, y, xb, yb, xl, yl, ax, ax0;
    std::vector<double> aty0, aty1, ax1;  // evaluation products
    std::vector<double> part;             // per-chunk reduction partials
    pdhg_params prm;
    std::vector<double> levels;
    double sigma_hat = 0, eta = 0, omega0 = 0, nb = 0, nc = 0;
    State st;
    std::vector<double> elog;
    int log_cap = 4096;
    std::vector<SnapCopy> snaps;
    bool initial_done = false;
    int status = PDHG_RUNNING;
    double t_setup = 0, t_iter = 0, t_start = 0;
    std::atomic<int> cancel{0};
};

namespace {

int fail(pdhg_cpu *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

// ---- parallel loops and deterministic reductions ----------------------

// f(r0, r1) over the thread row ranges of `cut`.
void par_rows(pdhg_cpu *c, const std::vector<int64_t> &cut,
              const std::function<void(int64_t, int64_t)> &f) {
    c->pool->run([&](int t) { f(cut[t], cut[t + 1]); });
}

// f(r0, r1) over [0, rows) cut into equal contiguous ranges per thread.
void par_range(pdhg_cpu *c, int64_t rows,
               const std::function<void(int64_t, int64_t)> &f) {
    const int T = c->pool->size();
    c->pool->run([&](int t) { f(rows * t / T, rows * (t + 1) / T); });
}

// Sum over [0, rows) of the `nq` quantities f(i, acc) adds into acc: fixed
// chunks of kChunk rows, partials added in chunk order (max for the entries
// flagged in is_max).  out[q] receives the totals.
void reduce_rows(pdhg_cpu *c, int64_t rows, int nq, const bool *is_max,
                 const std::function<void(int64_t, double *)> &f, double *out) {
    const int64_t nch = (rows + kChunk - 1) / kChunk;
    c->part.assign((size_t)std::max<int64_t>(nch, 1) * nq, 0.0);
    double *P = c->part.data();
    const int T = c->pool->size();
    c->pool->run([&](int t) {
        for (int64_t ch = nch * t / T; ch < nch * (t + 1) / T; ++ch) {
            double *acc = P + ch * nq;
            const int64_t r1 = std::min(rows, (ch + 1) * kChunk);
            for (int64_t i = ch * kChunk; i < r1; ++i) f(i, acc);
        }
    });
    for (int q = 0; q < nq; ++q) out[q] = 0.0;
    for (int64_t ch = 0; ch < nch; ++ch)
        for (int q = 0; q < nq; ++q) {
            const double v = P[ch * nq + q];
            out[q] = (is_max && is_max[q]) ? std::max(out[q], v) : out[q] + v;
        }
}

double dot(pdhg_cpu *c, const double *a, const double *b, int64_t k) {
    double s = 0.0;
    reduce_rows(c, k, 1, nullptr, [&](int64_t i, double *acc) { acc[0] += a[i] * b[i]; }, &s);
    return s;
}

// out = M v for the CSR (rp, ci, val) split by `cut`.
void spmv(pdhg_cpu *c, const std::vector<int64_t> &cut, const int64_t *rp,
          const int32_t *ci, const double *val, const double *v, double *out) {
    par_rows(c, cut, [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r) {
            double s = 0.0;
            for (int64_t p = rp[r]; p < rp[r + 1]; ++p) s += val[p] * v[ci[p]];
            out[r] = s;
        }
    });
}
void spmv_a(pdhg_cpu *c, const double *v, double *out) {
    spmv(c, c->cut_a, c->arp.data(), c->aci.data(), c->as.data(), v, out);
}
void spmv_at(pdhg_cpu *c, const double *v, double *out) {
    spmv(c, c->cut_at, c->atrp.data(), c->atci.data(), c->ats.data(), v, out);
}

// ---- setup ---------------------------------------------------------------

// Ruiz l_inf equilibration: `passes` simultaneous passes of
// D_r,i /= sqrt(max_j |a~_ij|), D_c,j /= sqrt(max_i |a~_ij|) with
// a~_ij = (D_r,i a_ij) D_c,j; a zero maximum counts as 1.
void ruiz(pdhg_cpu *c, int passes) {
    const int64_t m = c->m, n = c->n;
    c->dr.assign((size_t)m, 1.0);
    c->dc.assign((size_t)n, 1.0);
    std::vector<double> rho((size_t)m), kap((size_t)n);
    const int64_t *arp = c->arp.data(), *atrp = c->atrp.data();
    const int32_t *aci = c->aci.data(), *atci = c->atci.data();
    const double *av = c->av.data(), *atv = c->atv.data();
    for (int p = 0; p < passes; ++p) {
        const double *dr = c->dr.data(), *dc = c->dc.data();
        par_rows(c, c->cut_a, [&](int64_t r0, int64_t r1) {
            for (int64_t i = r0; i < r1; ++i) {
                double mx = 0.0;
                for (int64_t q = arp[i]; q < arp[i + 1]; ++q)
                    mx = std::max(mx, std::fabs((dr[i] * av[q]) * dc[aci[q]]));
                rho[i] = mx;
            }
        });
        par_rows(c, c->cut_at, [&](int64_t r0, int64_t r1) {
            for (int64_t j = r0; j < r1; ++j) {
                double mx = 0.0;
                for (int64_t q = atrp[j]; q < atrp[j + 1]; ++q)
                    mx = std::max(mx, std::fabs((dr[atci[q]] * atv[q]) * dc[j]));
                kap[j] = mx;
            }
        });
        par_range(c, m, [&](int64_t r0, int64_t r1) {
            for (int64_t i = r0; i < r1; ++i)
                c->dr[i] = c->dr[i] / std::sqrt(rho[i] == 0.0 ? 1.0 : rho[i]);
        });
        par_range(c, n, [&](int64_t r0, int64_t r1) {
            for (int64_t j = r0; j < r1; ++j)
                c->dc[j] = c->dc[j] / std::sqrt(kap[j] == 0.0 ? 1.0 : kap[j]);
        });
    }
}

// Scaled data from the factors: A~ (both CSRs), b~ = D_r b, c~ = D_c c,
// l~ = l / D_c, and the unscaled norms ||b||, ||c||.
void apply_scaling(pdhg_cpu *c) {
    const double *dr = c->dr.data(), *dc = c->dc.data();
    c->as.resize((size_t)c->nnz);
    c->ats.resize((size_t)c->nnz);
    par_rows(c, c->cut_a, [&](int64_t r0, int64_t r1) {
        for (int64_t i = r0; i < r1; ++i)
            for (int64_t q = c->arp[i]; q < c->arp[i + 1]; ++q) {
                const double a = (dr[i] * c->av[q]) * dc[c->aci[q]];
                c->as[q] = a;
                c->ats[c->perm[q]] = a;
            }
    });
    c->bs.resize((size_t)c->m);
    c->cs.resize((size_t)c->n);
    c->ls.assign((size_t)c->n, 0.0);
    for (int64_t i = 0; i < c->m; ++i) c->bs[i] = dr[i] * c->b0[i];
    for (int64_t j = 0; j < c->n; ++j) c->cs[j] = dc[j] * c->c0[j];
    if (c->has_l)
        for (int64_t j = 0; j < c->n; ++j) c->ls[j] = c->l0[j] / dc[j];
    c->nb = std::sqrt(dot(c, c->b0.data(), c->b0.data(), c->m));
    c->nc = std::sqrt(dot(c, c->c0.data(), c->c0.data(), c->n));
}

// sigma_hat ~ ||A~||_2: v0 = ones / sqrt(n), `iters` steps of
// w = A~^T A~ v, v = w / ||w||, then sqrt(||A~^T A~ v||).
double power_iteration(pdhg_cpu *c, int iters) {
    std::vector<double> v((size_t)c->n, 1.0 / std::sqrt((double)c->n)),
        u((size_t)c->m), w((size_t)c->n);
    double nw2 = 0.0;
    for (int it = 0; it <= iters; ++it) {
        spmv_a(c, v.data(), u.data());
        spmv_at(c, u.data(), w.data());
        nw2 = dot(c, w.data(), w.data(), c->n);
        if (it < iters) {
            const double nrm = std::sqrt(nw2);
            for (int64_t j = 0; j < c->n; ++j) v[j] = nrm > 0.0 ? w[j] / nrm : w[j];
        }
    }
    const double s = std::sqrt(std::sqrt(nw2));
    return (s > 0.0 && std::isfinite(s)) ? s : 1.0;
}

State fresh_state(pdhg_cpu *c) {
    State s;
    std::memset(&s, 0, sizeof s);
    const pdhg_params &p = c->prm;
    s.eta = c->eta;
    s.omega = c->omega0;
    s.tau = c->eta / c->omega0;
    s.sigma = c->eta * c->omega0;
    s.K_last = INFINITY;
    s.K_prev = INFINITY;
    s.nb = c->nb;
    s.nc = c->nc;
    s.eps_rel = p.eps_rel;
    s.beta_suff = p.beta_suff;
    s.beta_nec = p.beta_nec;
    s.beta_art = p.beta_art;
    s.omega_theta = p.omega_theta;
    s.omega_rule = p.omega_rule;
    s.pid_kp = p.pid_kp;
    s.pid_ki = p.pid_ki;
    s.pid_kd = p.pid_kd;
    s.stop_on = p.stop_on;
    s.variant = p.variant;
    s.reflect = p.reflect;
    s.status = PDHG_RUNNING;
    s.n_levels = (int)c->levels.size();
    s.literal = p.literal_snapshots;
    s.log_cap = c->log_cap;
    for (size_t i = 0; i < c->levels.size(); ++i) s.levels[i] = c->levels[i];
    return s;
}

void reset_iterate(pdhg_cpu *c) {
    for (auto *v : {&c->x, &c->xb, &c->xl, &c->aty0, &c->aty1})
        v->assign((size_t)c->n, 0.0);
    for (auto *v : {&c->y, &c->yb, &c->yl, &c->ax, &c->ax0, &c->ax1})
        v->assign((size_t)c->m, 0.0);
    c->st = fresh_state(c);
    c->elog.assign((size_t)c->log_cap * 8, 0.0);
    c->snaps.clear();
    c->initial_done = false;
    c->status = PDHG_RUNNING;
    c->t_iter = 0.0;
    c->cancel.store(0);
}

// ---- one iteration ---------------------------------------------------------

// t: the iteration's count since the last restart (from 1).
void iteration(pdhg_cpu *c, double t) {
    const State &s = c->st;
    const double tau = s.tau, sigma = s.sigma;
    const bool halpern = s.variant == 1, has_l = c->has_l;
    const double lam = t / (t + 1.0), rho = s.reflect;
    const int64_t *atrp = c->atrp.data(), *arp = c->arp.data();
    const int32_t *atci = c->atci.data(), *aci = c->aci.data();
    const double *ats = c->ats.data(), *as = c->as.data();
    double *x = c->x.data(), *y = c->y.data(), *xb = c->xb.data(), *yb = c->yb.data();
    double *ax = c->ax.data();
    const double *cs = c->cs.data(), *bs = c->bs.data(), *ls = c->ls.data();
    const double *xl = c->xl.data(), *yl = c->yl.data(), *ax0 = c->ax0.data();
    // primal half over rows j of A~^T (gathers y)
    par_rows(c, c->cut_at, [&](int64_t r0, int64_t r1) {
        for (int64_t j = r0; j < r1; ++j) {
            double g = 0.0;
            for (int64_t p = atrp[j]; p < atrp[j + 1]; ++p) g += ats[p] * y[atci[p]];
            const double v = x[j] - tau * (cs[j] - g);
            const double lj = has_l ? ls[j] : 0.0;
            const double xh = v < lj ? lj : v;
            if (halpern) {
                xb[j] = xh;     // T_x(z), gathered by the dual half
                x[j] = lam * ((1.0 + rho) * xh - rho * x[j]) + (1.0 - lam) * xl[j];
            } else {
                x[j] = xh;
                xb[j] = xb[j] + (xh - xb[j]) / t;
            }
        }
    });
    // dual half over rows i of A~ (gathers the new x, or T_x(z))
    const double *xg = halpern ? xb : x;
    par_rows(c, c->cut_a, [&](int64_t r0, int64_t r1) {
        for (int64_t i = r0; i < r1; ++i) {
            double q = 0.0;
            for (int64_t p = arp[i]; p < arp[i + 1]; ++p) q += as[p] * xg[aci[p]];
            const double yh = y[i] + sigma * (bs[i] - ((q + q) - ax[i]));
            if (halpern) {
                y[i] = lam * ((1.0 + rho) * yh - rho * y[i]) + (1.0 - lam) * yl[i];
                ax[i] = lam * ((1.0 + rho) * q - rho * ax[i]) + (1.0 - lam) * ax0[i];
            } else {
                y[i] = yh;
                ax[i] = q;
                yb[i] = yb[i] + (yh - yb[i]) / t;
            }
        }
    });
}

// ---- evaluation --------------------------------------------------------------

// The FP64 evaluation after `batch` iterations (initial: the k = 0 check):
// candidate products, reduction totals, control_decide, then the snapshot
// copies and the restart the decisions ask for.
void evaluate(pdhg_cpu *c, int batch, bool initial) {
    const int64_t m = c->m, n = c->n;
    const bool halpern = c->st.variant == 1;
    const int ncand = (initial && !halpern) ? 1 : 2;
    const double *ls = c->ls.data();
    // products: candidate 0 uses the stored A~ x; candidate 1 is the average,
    // or T(z) formed here in FP64
    spmv_at(c, c->y.data(), c->aty0.data());
    if (halpern) {
        const double tau = c->st.tau, sigma = c->st.sigma;
        par_range(c, n, [&](int64_t r0, int64_t r1) {
            for (int64_t j = r0; j < r1; ++j) {
                const double v = c->x[j] - tau * (c->cs[j] - c->aty0[j]);
                const double lj = c->has_l ? ls[j] : 0.0;
                c->xb[j] = v < lj ? lj : v;
            }
        });
        spmv_a(c, c->xb.data(), c->ax1.data());
        par_range(c, m, [&](int64_t r0, int64_t r1) {
            for (int64_t i = r0; i < r1; ++i) {
                const double q = c->ax1[i];
                c->yb[i] = c->y[i] + sigma * (c->bs[i] - ((q + q) - c->ax[i]));
            }
        });
        spmv_at(c, c->yb.data(), c->aty1.data());
    } else if (!initial) {
        spmv_a(c, c->xb.data(), c->ax1.data());
        spmv_at(c, c->yb.data(), c->aty1.data());
    }
    const double *X[2] = {c->x.data(), c->xb.data()}, *Y[2] = {c->y.data(), c->yb.data()};
    const double *AX[2] = {c->ax.data(), c->ax1.data()};
    const double *ATY[2] = {c->aty0.data(), c->aty1.data()};
    const double *bs = c->bs.data(), *cs = c->cs.data(), *dr = c->dr.data(),
                 *dc = c->dc.data(), *xl = c->xl.data(), *yl = c->yl.data();
    constexpr int NQ = 2 * Q_NQ;
    bool is_max[NQ] = {false};
    for (int cc = 0; cc < 2; ++cc) {
        is_max[cc * Q_NQ + Q_RPMAX] = true;
        is_max[cc * Q_NQ + Q_RDMAX] = true;
    }
    double tr[NQ], tc[NQ];
    // rows: primal residual, b^T y, distance of y from the restart point
    reduce_rows(c, m, NQ, is_max, [&](int64_t i, double *acc) {
        for (int cc = 0; cc < ncand; ++cc) {
            double *a = acc + cc * Q_NQ;
            const double rs = bs[i] - AX[cc][i];
            const double ru = rs / dr[i];
            a[Q_RP2] += ru * ru;
            a[Q_RPMAX] = std::max(a[Q_RPMAX], std::fabs(ru));
            a[Q_SRP2] += rs * rs;
            a[Q_BY] += bs[i] * Y[cc][i];
            const double d = Y[cc][i] - yl[i];
            a[Q_DY2] += d * d;
        }
        if (ncand > 1) {
            const double f = Y[1][i] - Y[0][i];
            acc[Q_NQ + Q_FY2] += f * f;
        }
    }, tr);
    // columns: dual residual with z = max(0, c - A^T y), c^T x, l^T z,
    // distance of x from the restart point
    reduce_rows(c, n, NQ, is_max, [&](int64_t j, double *acc) {
        const double lj = c->has_l ? ls[j] : 0.0;
        for (int cc = 0; cc < ncand; ++cc) {
            double *a = acc + cc * Q_NQ;
            const double ds = cs[j] - ATY[cc][j];
            const double zs = ds > 0.0 ? ds : 0.0;
            const double rds = zs - ds;
            const double du = ds / dc[j];
            const double zu = du > 0.0 ? du : 0.0;
            const double rdu = zu - du;
            a[Q_RD2] += rdu * rdu;
            a[Q_RDMAX] = std::max(a[Q_RDMAX], std::fabs(rdu));
            a[Q_SRD2] += rds * rds;
            a[Q_CX] += cs[j] * X[cc][j];
            a[Q_LZ] += lj * zs;
            const double d = X[cc][j] - xl[j];
            a[Q_DX2] += d * d;
        }
        if (ncand > 1) {
            const double f = X[1][j] - X[0][j];
            acc[Q_NQ + Q_FX2] += f * f;
        }
    }, tc);
    double tot[2][Q_NQ];
    for (int cc = 0; cc < 2; ++cc)
        for (int q = 0; q < Q_NQ; ++q) {
            const double a = tr[cc * Q_NQ + q], b = tc[cc * Q_NQ + q];
            tot[cc][q] = (q == Q_RPMAX || q == Q_RDMAX) ? std::max(a, b) : a + b;
        }
    State &s = c->st;
    control_decide(&s, tot, ncand, batch, initial ? 1 : 0, c->elog.data());
    // snapshots of the chosen candidate, unscaled
    if (s.snap_n > 0) {
        const int cd = s.snap_cand;
        for (int q = 0; q < s.snap_n; ++q) {
            const int idx = s.snap_first + q;
            SnapCopy sc;
            std::memset(&sc.info, 0, sizeof sc.info);
            sc.info.level = s.snap_level[idx];
            sc.info.iter = s.snap_iter[idx];
            sc.info.maxresid = s.snap_mr[idx];
            sc.info.candidate = s.snap_cand_of[idx];
            sc.info.t_wall = now_s() - c->t_start;
            sc.x.resize((size_t)n);
            sc.y.resize((size_t)m);
            sc.z.resize((size_t)n);
            for (int64_t j = 0; j < n; ++j) {
                sc.x[j] = dc[j] * X[cd][j];
                const double d = (cs[j] - ATY[cd][j]) / dc[j];
                sc.z[j] = d > 0.0 ? d : 0.0;
            }
            for (int64_t i = 0; i < m; ++i) sc.y[i] = dr[i] * Y[cd][i];
            c->snaps.push_back(std::move(sc));
        }
    }
    // restart or final copy of a candidate into the current iterate
    if (s.copy_pending) {
        const bool avg = s.copy_avg != 0, last = s.set_last != 0;
        par_range(c, n, [&](int64_t r0, int64_t r1) {
            for (int64_t j = r0; j < r1; ++j) {
                const double v = avg ? c->xb[j] : c->x[j];
                if (avg) c->x[j] = v;
                if (last) {
                    c->xl[j] = v;
                    c->xb[j] = 0.0;
                }
            }
        });
        par_range(c, m, [&](int64_t r0, int64_t r1) {
            for (int64_t i = r0; i < r1; ++i) {
                const double v = avg ? c->yb[i] : c->y[i];
                if (avg) {
                    c->y[i] = v;
                    c->ax[i] = c->ax1[i];
                }
                if (last) {
                    c->yl[i] = v;
                    c->yb[i] = 0.0;
                    if (halpern) c->ax0[i] = avg ? c->ax1[i] : c->ax[i];
                }
            }
        });
    }
}

// Relative KKT of the current iterate (candidate 0) on the unscaled data.
void kkt_current(pdhg_cpu *c, pdhg_kkt *o) {
    std::memset(o, 0, sizeof *o);
    // recomputed for the current iterate (the evaluation's statistics may
    // predate the copy of the returned candidate into it)
    std::vector<double> aty((size_t)c->n), ax((size_t)c->m);
    spmv_at(c, c->y.data(), aty.data());
    spmv_a(c, c->x.data(), ax.data());
    double rp2 = 0, rpm = 0, by = 0, rd2 = 0, rdm = 0, cx = 0, lz = 0;
    for (int64_t i = 0; i < c->m; ++i) {
        const double ru = (c->bs[i] - ax[i]) / c->dr[i];
        rp2 += ru * ru;
        rpm = std::max(rpm, std::fabs(ru));
        by += c->bs[i] * c->y[i];
    }
    for (int64_t j = 0; j < c->n; ++j) {
        const double ds = c->cs[j] - aty[j];
        const double zs = ds > 0.0 ? ds : 0.0;
        const double du = ds / c->dc[j];
        const double zu = du > 0.0 ? du : 0.0;
        rd2 += (zu - du) * (zu - du);
        rdm = std::max(rdm, std::fabs(zu - du));
        cx += c->cs[j] * c->x[j];
        lz += (c->has_l ? c->ls[j] : 0.0) * zs;
    }
    o->norm_rp = std::sqrt(rp2);
    o->norm_rd = std::sqrt(rd2);
    o->rp_inf = rpm;
    o->rd_inf = rdm;
    o->pobj = cx;
    o->dobj = by + lz;
    o->rel_p = o->norm_rp / (1.0 + c->nb);
    o->rel_d = o->norm_rd / (1.0 + c->nc);
    o->rel_gap = std::fabs(o->pobj - o->dobj) / (1.0 + std::fabs(o->pobj) + std::fabs(o->dobj));
    o->maxresid = std::max(o->rel_p, std::max(o->rel_d, o->rel_gap));
    o->iter = c->st.k;
}

}  // namespace

// ============================================================== the C ABI

extern "C" {

const char *pdhg_cpu_last_error(const pdhg_cpu *c) {
    return c ? c->err.c_str() : "null context";
}

int pdhg_cpu_create(int threads, pdhg_cpu **out) {
    if (!out || threads < 1 || threads > 1024) return PDHG_E_ARG;
    *out = nullptr;
    try {
        pdhg_cpu *c = new pdhg_cpu();
        c->pool.reset(new Pool(threads));
        pdhg_params_default(&c->prm);
        *out = c;
    } catch (...) {
        return PDHG_E_OOM;
    }
    return PDHG_OK;
}

void pdhg_cpu_destroy(pdhg_cpu *c) { delete c; }

int pdhg_cpu_set_threads(pdhg_cpu *c, int threads) {
    if (!c || threads < 1 || threads > 1024) return fail(c, PDHG_E_ARG, "bad thread count");
    try {
        c->pool.reset();
        c->pool.reset(new Pool(threads));
        if (c->loaded) {
            c->cut_a = split_rows(c->m, c->arp.data(), threads);
            c->cut_at = split_rows(c->n, c->atrp.data(), threads);
        }
    } catch (...) {
        return fail(c, PDHG_E_OOM, "thread pool");
    }
    return PDHG_OK;
}

int pdhg_cpu_load(pdhg_cpu *c, int64_t m, int64_t n, int64_t nnz,
                  const int64_t *a_rp, const int32_t *a_ci, const double *a_v,
                  const int64_t *at_rp, const int32_t *at_ci,
                  const double *at_v, const double *b, const double *cv,
                  const double *lb) {
    if (!c) return PDHG_E_ARG;
    c->err.clear();
    if (m < 1 || n < 1 || nnz < 0 || !a_rp || !at_rp || !b || !cv ||
        (nnz > 0 && (!a_ci || !a_v || !at_ci || !at_v)))
        return fail(c, PDHG_E_ARG, "bad argument to pdhg_cpu_load");
    try {
        std::vector<int64_t> perm((size_t)nnz);
        char msg[256] = {0};
        const int rc = pdhg_check_transpose(m, n, nnz, a_rp, a_ci, a_v, at_rp,
                                            at_ci, at_v, perm.data(), msg, sizeof msg);
        if (rc != PDHG_OK) return fail(c, rc, msg);
        c->loaded = c->configured = false;
        c->m = m;
        c->n = n;
        c->nnz = nnz;
        c->arp.assign(a_rp, a_rp + m + 1);
        c->atrp.assign(at_rp, at_rp + n + 1);
        c->aci.assign(a_ci, a_ci + nnz);
        c->atci.assign(at_ci, at_ci + nnz);
        c->av.assign(a_v, a_v + nnz);
        c->atv.assign(at_v, at_v + nnz);
        c->perm.swap(perm);
        c->b0.assign(b, b + m);
        c->c0.assign(cv, cv + n);
        c->has_l = lb != nullptr;
        if (c->has_l) c->l0.assign(lb, lb + n);
        else c->l0.clear();
        const int T = c->pool->size();
        c->cut_a = split_rows(m, c->arp.data(), T);
        c->cut_at = split_rows(n, c->atrp.data(), T);
        c->loaded = true;
    } catch (...) {
        return fail(c, PDHG_E_OOM, "host allocation failed");
    }
    return PDHG_OK;
}

int pdhg_cpu_configure(pdhg_cpu *c, const pdhg_params *p) {
    if (!c) return PDHG_E_ARG;
    c->err.clear();
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    if (!p) return fail(c, PDHG_E_ARG, "null params");
    if (p->precision != PDHG_FP64)
        return fail(c, PDHG_E_ARG, "the CPU PDHG computes in FP64 only");
    if (p->polish) return fail(c, PDHG_E_ARG, "no feasibility polishing on the CPU PDHG");
    if (p->eval_every < 1 || p->ruiz_passes < 0 || p->power_iters < 0 ||
        p->n_levels < 0 || p->n_levels > kMaxLevels || (p->n_levels > 0 && !p->levels) ||
        !(p->eps_rel >= 0.0) || p->max_iters < 0 || (p->variant != 0 && p->variant != 1) ||
        !(p->reflect >= 0.0 && p->reflect <= 1.0) ||
        (p->omega_rule != 0 && p->omega_rule != 1) || p->stop_on < 0 || p->stop_on > 2)
        return fail(c, PDHG_E_ARG, "invalid parameters");
    for (int i = 1; i < p->n_levels; ++i)
        if (!(p->levels[i] < p->levels[i - 1]))
            return fail(c, PDHG_E_ARG, "snapshot levels must be strictly descending");
    try {
        const double t0 = now_s();
        c->prm = *p;
        c->levels.assign(p->levels, p->levels + p->n_levels);
        c->prm.levels = nullptr;
        ruiz(c, p->ruiz_passes);
        apply_scaling(c);
        c->sigma_hat = 0.0;
        if (p->eta > 0.0) {
            c->eta = p->eta;
        } else {
            c->sigma_hat = power_iteration(c, p->power_iters);
            c->eta = p->eta_factor / c->sigma_hat;
        }
        const double nbs = std::sqrt(dot(c, c->bs.data(), c->bs.data(), c->m));
        const double ncs = std::sqrt(dot(c, c->cs.data(), c->cs.data(), c->n));
        if (p->omega0 > 0.0)
            c->omega0 = p->omega0;
        else
            c->omega0 = (nbs > 1e-10 && ncs > 1e-10) ? ncs / nbs : 1.0;
        reset_iterate(c);
        c->configured = true;
        c->t_setup = now_s() - t0;
    } catch (...) {
        return fail(c, PDHG_E_OOM, "host allocation failed");
    }
    return PDHG_OK;
}

int pdhg_cpu_iterate(pdhg_cpu *c, int64_t max_iters, int *status) {
    if (!c) return PDHG_E_ARG;
    c->err.clear();
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    if (max_iters < 0) return fail(c, PDHG_E_ARG, "negative iteration count");
    try {
        State &s = c->st;
        if (!c->initial_done) {
            c->t_start = now_s();
            evaluate(c, 0, true);
            c->initial_done = true;
            c->status = s.status;
        }
        const double t0 = now_s();
        const int64_t limit = c->prm.max_iters;
        const int64_t target = std::min<int64_t>((int64_t)s.k + max_iters, limit);
        const int N = c->prm.eval_every;
        while (c->status == PDHG_RUNNING) {
            if ((int64_t)s.k >= limit) {
                s.status = c->status = PDHG_ITER_LIMIT;
                break;
            }
            if ((int64_t)s.k >= target) break;
            const int64_t to_eval = N - (int64_t)s.k % N;
            const int64_t B = std::min<int64_t>(target - (int64_t)s.k, to_eval);
            for (int64_t off = 0; off < B; ++off)
                iteration(c, (double)(s.t_base + off + 1));
            if (B == to_eval) {
                evaluate(c, (int)B, false);
                c->status = s.status;
                if (c->status == PDHG_RUNNING) {
                    if (c->cancel.load()) s.status = c->status = PDHG_CANCELLED;
                    else if (c->prm.time_limit_s > 0 && now_s() - c->t_start > c->prm.time_limit_s)
                        s.status = c->status = PDHG_TIME_LIMIT;
                }
            } else {
                s.k += B;
                s.t_base += B;
            }
        }
        c->t_iter += now_s() - t0;
        if (status) *status = c->status;
    } catch (...) {
        return fail(c, PDHG_E_OOM, "host allocation failed");
    }
    return PDHG_OK;
}

int pdhg_cpu_cancel(pdhg_cpu *c) {
    if (!c) return PDHG_E_ARG;
    c->cancel.store(1);
    return PDHG_OK;
}

int pdhg_cpu_get_info(pdhg_cpu *c, pdhg_info *o) {
    if (!c || !o) return PDHG_E_ARG;
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    std::memset(o, 0, sizeof *o);
    const State &s = c->st;
    o->status = c->status;
    o->candidate = s.returned_cand;
    o->iters = s.k;
    o->restarts = s.restarts;
    o->n_snap = (int)c->snaps.size();
    o->sigma_hat = c->sigma_hat;
    o->eta = c->eta;
    o->omega0 = c->omega0;
    o->omega = s.omega;
    o->tau = s.tau;
    o->sigma = s.sigma;
    o->t_setup = c->t_setup;
    o->t_iter = c->t_iter;
    try {
        kkt_current(c, &o->kkt);
    } catch (...) {
        return fail(c, PDHG_E_OOM, "host allocation failed");
    }
    return PDHG_OK;
}

int pdhg_cpu_get_iterate(pdhg_cpu *c, double *x, double *y, double *z) {
    if (!c) return PDHG_E_ARG;
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    try {
        std::vector<double> aty((size_t)c->n);
        if (z) spmv_at(c, c->y.data(), aty.data());
        for (int64_t j = 0; j < c->n; ++j) {
            if (x) x[j] = c->dc[j] * c->x[j];
            if (z) {
                const double d = (c->cs[j] - aty[j]) / c->dc[j];
                z[j] = d > 0.0 ? d : 0.0;
            }
        }
        if (y)
            for (int64_t i = 0; i < c->m; ++i) y[i] = c->dr[i] * c->y[i];
    } catch (...) {
        return fail(c, PDHG_E_OOM, "host allocation failed");
    }
    return PDHG_OK;
}

int pdhg_cpu_get_scaling(pdhg_cpu *c, double *dr, double *dc) {
    if (!c) return PDHG_E_ARG;
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    if (dr) std::copy(c->dr.begin(), c->dr.end(), dr);
    if (dc) std::copy(c->dc.begin(), c->dc.end(), dc);
    return PDHG_OK;
}

int pdhg_cpu_eval_log(pdhg_cpu *c, double *out, int cap, int *count) {
    if (!c) return PDHG_E_ARG;
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    const int nlog = c->st.n_log;
    if (count) *count = nlog;
    const int k = std::min(nlog, std::max(cap, 0));
    if (out && k > 0) std::copy(c->elog.begin(), c->elog.begin() + 8 * k, out);
    return PDHG_OK;
}

int pdhg_cpu_snapshot_count(pdhg_cpu *c, int *count) {
    if (!c || !count) return PDHG_E_ARG;
    *count = (int)c->snaps.size();
    return PDHG_OK;
}

int pdhg_cpu_snapshot(pdhg_cpu *c, int idx, pdhg_snapshot_info *info, double *x,
                      double *y, double *z) {
    if (!c) return PDHG_E_ARG;
    if (idx < 0 || idx >= (int)c->snaps.size())
        return fail(c, PDHG_E_ARG, "snapshot index out of range");
    const SnapCopy &s = c->snaps[idx];
    if (info) *info = s.info;
    if (x) std::copy(s.x.begin(), s.x.end(), x);
    if (y) std::copy(s.y.begin(), s.y.end(), y);
    if (z) std::copy(s.z.begin(), s.z.end(), z);
    return PDHG_OK;
}

int pdhg_cpu_stream_bw(int threads, int64_t bytes, int reps, double *gb_s) {
    if (threads < 1 || threads > 1024 || bytes < (1 << 20) || reps < 1 || !gb_s)
        return PDHG_E_ARG;
    try {
        const int64_t k = bytes / 8;
        std::vector<double> a((size_t)k);
        Pool pool(threads);
        // first touch by the thread that reads each part
        pool.run([&](int t) {
            for (int64_t i = k * t / threads; i < k * (t + 1) / threads; ++i) a[i] = 1.0;
        });
        std::vector<double> sink((size_t)threads * 8, 0.0);
        auto pass = [&](int t) {
            double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
            const int64_t r0 = k * t / threads, r1 = k * (t + 1) / threads;
            int64_t i = r0;
            for (; i + 4 <= r1; i += 4) {
                s0 += a[i];
                s1 += a[i + 1];
                s2 += a[i + 2];
                s3 += a[i + 3];
            }
            for (; i < r1; ++i) s0 += a[i];
            sink[(size_t)t * 8] += (s0 + s1) + (s2 + s3);
        };
        pool.run(pass);                    // warm-up
        const double t0 = now_s();
        for (int r = 0; r < reps; ++r) pool.run(pass);
        const double dt = now_s() - t0;
        *gb_s = dt > 0 ? (double)k * 8.0 * reps / dt / 1e9 : 0.0;
        volatile double keep = sink[0];
        (void)keep;
    } catch (...) {
        return PDHG_E_OOM;
    }
    return PDHG_OK;
}

}  // extern "C"
