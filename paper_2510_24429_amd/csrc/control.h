// control.h -- the decisions of one KKT evaluation, shared by the GPU
// control kernel (one thread) and the CPU PDHG.
//
// Input: per candidate (0 the current iterate; 1 the average, or T(z) for the
// reflected Halpern iteration) the totals of the reduction quantities Q_*
// over the rows and columns.  The function forms the relative KKT errors of
// Section 2 (maxresid is their maximum, Algorithm 1's test quantity), runs
// Algorithm 1's snapshot test on the better candidate, the eps_rel stop and
// the adaptive restart with its primal-weight update, and appends one record
// to the evaluation log.  What it decides for the iterate (copy a candidate
// into it, make it the restart point) it leaves in the State for the caller
// to apply.
#pragma once

#include <cmath>

#include "internal.h"

#if defined(__HIPCC__)
#define PDHG_HD __host__ __device__
#else
#define PDHG_HD
#endif

namespace pdhg {

PDHG_HD inline double kkt_w(const double *S, double w) {
    return sqrt(w * w * S[S_SP2] + S[S_SD2] / (w * w) + S[S_SG] * S[S_SG]);
}

// The measure a solve stops on and picks its candidate by: maxresid, or for
// a feasibility phase the relative primal (1) or dual (2) residual alone.
PDHG_HD inline double stop_metric(const State *st, const double *S) {
    return st->stop_on == 1 ? S[S_RELP] : st->stop_on == 2 ? S[S_RELD] : S[S_MAXR];
}

// Primal weight at a restart from the distances dx, dy travelled since the
// previous restart: smoothing toward dy / dx in log space (omega_rule 0), or
// PID control of log omega on the error e = log(omega dx / dy) (rule 1).
// Unchanged when either distance is below 1e-10.
PDHG_HD inline double omega_update(State *st, double om, double dx, double dy) {
    if (!(dx > 1e-10 && dy > 1e-10)) return om;
    if (st->omega_rule == 1) {
        const double e = log(om * dx / dy);
        st->pid_int += e;
        const double lw = log(om) - (st->pid_kp * e + st->pid_ki * st->pid_int +
                                     st->pid_kd * (e - st->pid_eprev));
        st->pid_eprev = e;
        return exp(lw);
    }
    return exp(st->omega_theta * log(dy / dx) + (1.0 - st->omega_theta) * log(om));
}

// The decisions after `batch` iterations (initial: the k = 0 check of the
// starting point), in this order: statistics of both candidates, Algorithm
// 1's snapshot test on the better one, the eps_rel stop, then the adaptive
// restart on KKT_omega.  tot[c][q]: totals of candidate c, ncand of them.
PDHG_HD inline void control_decide(State *st, const double (*tot)[Q_NQ],
                                   int ncand, int batch, int initial,
                                   double *elog) {
    st->k += batch;
    st->t_base += batch;
    const long long k = st->k, t = st->t_base;
    double om = st->omega;
    bool finite = true;
    for (int c = 0; c < ncand; ++c) {
        double *S = st->stats[c];
        const double *Q = tot[c];
        S[S_NRP] = sqrt(Q[Q_RP2]);
        S[S_NRD] = sqrt(Q[Q_RD2]);
        S[S_RPINF] = Q[Q_RPMAX];
        S[S_RDINF] = Q[Q_RDMAX];
        S[S_POBJ] = Q[Q_CX];
        S[S_DOBJ] = Q[Q_BY] + Q[Q_LZ];
        S[S_RELP] = S[S_NRP] / (1.0 + st->nb);
        S[S_RELD] = S[S_NRD] / (1.0 + st->nc);
        S[S_RELG] = fabs(S[S_POBJ] - S[S_DOBJ]) /
                    (1.0 + fabs(S[S_POBJ]) + fabs(S[S_DOBJ]));
        double mr = S[S_RELP];
        if (S[S_RELD] > mr) mr = S[S_RELD];
        if (S[S_RELG] > mr) mr = S[S_RELG];
        S[S_SP2] = Q[Q_SRP2];
        S[S_SD2] = Q[Q_SRD2];
        S[S_SG] = Q[Q_CX] - Q[Q_BY] - Q[Q_LZ];
        S[S_DX2] = Q[Q_DX2];
        S[S_DY2] = Q[Q_DY2];
        const bool f = __builtin_isfinite(S[S_RELP]) && __builtin_isfinite(S[S_RELD]) &&
                       __builtin_isfinite(S[S_RELG]) && __builtin_isfinite(S[S_SP2]) &&
                       __builtin_isfinite(S[S_SD2]) && __builtin_isfinite(S[S_SG]);
        S[S_MAXR] = f ? mr : NAN;
        S[S_FIN] = f ? 1.0 : 0.0;
        finite = finite && f;
    }
    st->last_ncand = ncand;
    st->copy_pending = 0;
    st->copy_avg = 0;
    st->set_last = 0;
    st->snap_n = 0;
    st->polish_due = 0;

    if (st->variant == 1) {
        // reflected Halpern: candidate 1 is T(z); z itself is not projected,
        // so T(z) is the reported point; restarts test ||z - T(z)||_omega
        const double fx2 = tot[1][Q_FX2], fy2 = tot[1][Q_FY2];
        st->fx2 = fx2;
        st->fy2 = fy2;
        const double r_cur = sqrt(om * fx2 + fy2 / om);
        int restarted = 0;
        if (!finite || !__builtin_isfinite(r_cur)) {
            st->status = PDHG_NUMERICAL;
        } else {
            const double mrb = st->stats[1][S_MAXR];
            int fired = 0;
            const int first = st->snap_count;
            while (st->next_level < st->n_levels && mrb <= st->levels[st->next_level]) {
                const int s = st->snap_count;
                st->snap_level[s] = st->levels[st->next_level];
                st->snap_iter[s] = k;
                st->snap_mr[s] = mrb;
                st->snap_cand_of[s] = 1;
                ++st->snap_count;
                ++st->next_level;
                ++fired;
                if (st->literal) break;
            }
            if (fired) {
                st->snap_first = first;
                st->snap_n = fired;
                st->snap_cand = 1;
            }
            if (stop_metric(st, st->stats[1]) <= st->eps_rel) {
                st->status = PDHG_CONVERGED;
                st->returned_cand = 1;
                st->copy_pending = 1;
                st->copy_avg = 1;
            } else if (initial) {
                st->K_last = r_cur;
            } else {
                // a polishing attempt is decided on T(z) before a restart
                st->polish_due = st->polish && st->stats[1][S_RELG] <= st->eps_rel &&
                                 k >= st->next_polish;
                st->polish_cand = 1;
                const bool r = (r_cur <= st->beta_suff * st->K_last) ||
                               (r_cur <= st->beta_nec * st->K_last && r_cur > st->K_prev) ||
                               ((double)t >= st->beta_art * (double)k);
                if (r) {
                    const double *S = st->stats[1];
                    om = omega_update(st, om, sqrt(S[S_DX2]), sqrt(S[S_DY2]));
                    st->omega = om;
                    st->tau = st->eta / om;
                    st->sigma = st->eta * om;
                    st->copy_pending = 1;
                    st->copy_avg = 1;
                    st->set_last = 1;
                    st->t_base = 0;
                    st->K_last = sqrt(om * fx2 + fy2 / om);
                    st->K_prev = INFINITY;
                    ++st->restarts;
                    restarted = 1;
                } else {
                    st->K_prev = r_cur;
                }
            }
        }
        if (elog && st->n_log < st->log_cap) {
            double *e = elog + 8 * st->n_log;
            e[0] = (double)k;
            e[1] = st->stats[0][S_MAXR];
            e[2] = st->stats[1][S_MAXR];
            e[3] = r_cur;
            e[4] = st->K_last;
            e[5] = (double)restarted;
            e[6] = 1.0;
            e[7] = om;
            ++st->n_log;
        }
        return;
    }

    const int best = (ncand > 1 && stop_metric(st, st->stats[1]) <
                                       stop_metric(st, st->stats[0])) ? 1 : 0;
    double Kcur = kkt_w(st->stats[0], om);
    double Kavg = ncand > 1 ? kkt_w(st->stats[1], om) : INFINITY;
    int restarted = 0, cand = (Kavg < Kcur) ? 1 : 0;
    if (initial) st->K_last = Kcur;

    if (!finite) {
        st->status = PDHG_NUMERICAL;
    } else {
        const double mrb = st->stats[best][S_MAXR];
        int fired = 0;
        const int first = st->snap_count;
        while (st->next_level < st->n_levels && mrb <= st->levels[st->next_level]) {
            const int s = st->snap_count;
            st->snap_level[s] = st->levels[st->next_level];
            st->snap_iter[s] = k;
            st->snap_mr[s] = mrb;
            st->snap_cand_of[s] = best;
            ++st->snap_count;
            ++st->next_level;
            ++fired;
            if (st->literal) break;
        }
        if (fired) {
            st->snap_first = first;
            st->snap_n = fired;
            st->snap_cand = best;
        }
        if (stop_metric(st, st->stats[best]) <= st->eps_rel) {
            st->status = PDHG_CONVERGED;
            st->returned_cand = best;
            if (best == 1) {
                st->copy_pending = 1;
                st->copy_avg = 1;
            }
        } else if (!initial) {
            // a polishing attempt is decided on the better candidate before
            // the restart test may replace it
            st->polish_due = st->polish && st->stats[best][S_RELG] <= st->eps_rel &&
                             k >= st->next_polish;
            st->polish_cand = best;
            const double *S = st->stats[cand];
            const double Kc = cand ? Kavg : Kcur;
            const bool r = (Kc <= st->beta_suff * st->K_last) ||
                           (Kc <= st->beta_nec * st->K_last && Kc > st->K_prev) ||
                           ((double)t >= st->beta_art * (double)k);
            if (r) {
                om = omega_update(st, om, sqrt(S[S_DX2]), sqrt(S[S_DY2]));
                st->omega = om;
                st->tau = st->eta / om;
                st->sigma = st->eta * om;
                st->copy_pending = 1;
                st->copy_avg = cand;
                st->set_last = 1;
                st->t_base = 0;
                st->K_last = kkt_w(S, om);
                st->K_prev = INFINITY;
                ++st->restarts;
                restarted = 1;
            } else {
                st->K_prev = Kc;
            }
        }
    }
    if (elog && st->n_log < st->log_cap) {
        double *e = elog + 8 * st->n_log;
        e[0] = (double)k;
        e[1] = st->stats[0][S_MAXR];
        e[2] = ncand > 1 ? st->stats[1][S_MAXR] : NAN;
        e[3] = Kcur;
        e[4] = Kavg;
        e[5] = (double)restarted;
        e[6] = (double)cand;
        e[7] = om;
        ++st->n_log;
    }
}

}  // namespace pdhg
