"""Pins of the oracle's PDHG internals against numpy restatements.

The paper leaves the iteration's internals to the cuPDLP+ line of work, so
the oracle's step, averages, weighted KKT error, restart rule, primal-weight
update and Halpern schedule are readings.  These tests replay each reading
in dense numpy (tests/replay.py) from the oracle's own traced iterates, Ruiz
factors and evaluation log, one step or one decision at a time, and require:

  - every traced iterate is one PDHG step (or one Halpern step) of the
    previous one, with tau = eta / w and sigma = eta w for the weight w in
    force;
  - the average at an evaluation is the arithmetic mean of the iterates
    produced since the last restart (the restart point itself excluded);
  - the logged maxresid of both candidates and the logged weighted KKT
    errors (or, for the Halpern variant, the fixed-point residuals) equal
    the recomputed ones;
  - every logged restart flag and candidate is the beta 0.2 / 0.8 / 0.36 rule
    applied to the recomputed sequence, and the weight after each restart is
    the smoothed (or PID) update of the recomputed distances;
  - Algorithm 1's snapshots fire at the first evaluation whose recomputed
    maxresid reaches the level.

A decision whose recomputed margin is within 1e-9 (relative) of its
threshold would not pin anything; the tests assert that none occurs.
"""
import numpy as np
import pytest

from paper_2510_24429_amd import lpgen
from tests import replay as R

TIE = 1e-9


def _margin_ok(a, b):
    return abs(a - b) > TIE * max(abs(a), abs(b), 1e-300)


def _start(S, x0, y0):
    if x0 is None:
        return np.zeros(S.A.shape[1]), np.zeros(S.A.shape[0])
    return R.to_scaled(S, x0, y0)


def replay_averaged(oracle, lp, E, T, l=None, x0=None, y0=None, omega_rule=0,
                    pid=(0.99, 0.01, 0.0), beta=(0.2, 0.8, 0.36), **kw):
    """Run the averaged variant for T iterations (never stopping) and replay
    it; returns (list of (k, reason, cand) for every restart, eval records)."""
    r = oracle.solve(lp, l=l, x0=x0, y0=y0, eps_rel=1e-30, max_iters=T,
                     trace_k=T, eval_every=E, omega_rule=omega_rule,
                     pid_kp=pid[0], pid_ki=pid[1], pid_kd=pid[2],
                     beta_suff=beta[0], beta_nec=beta[1], beta_art=beta[2], **kw)
    assert r.info["status"] == 2 and r.info["iters"] == T
    dr, dc, _ = oracle.ruiz(lp, 10)
    S = R.scaled(lp, dr, dc, l)
    eta, omega = r.info["eta"], r.info["omega0"]
    log = r.eval_log
    assert log.shape[0] == T // E + 1
    X = r.trace_x / dc[None, :]
    Y = r.trace_y / dr[None, :]
    xs, ys = _start(S, x0, y0)
    xl, yl = xs.copy(), ys.copy()
    # k = 0: the starting point alone, no restart
    m0 = R.kkt(S, *R.to_unscaled(S, xs, ys))["maxresid"]
    assert R.close(log[0, 1], m0, 1e-10, 1e-14)
    K_last = R.kkt_omega(S, xs, ys, omega)
    assert R.close(log[0, 3], K_last, 1e-10, 1e-14)
    K_prev = np.inf
    pid_int, pid_eprev = 0.0, 0.0
    hist_x, hist_y = [], []
    last_k = 0
    restarts, records = [], []
    for k in range(1, T + 1):
        tau, sigma = eta / omega, eta * omega
        xr, yr = R.pdhg_step(S, xs, ys, tau, sigma)
        hist_x.append(xr)
        hist_y.append(yr)
        xs, ys = X[k - 1], Y[k - 1]          # the oracle's (post-evaluation) iterate
        if k % E:
            assert R.close(xs, xr, 1e-12, 1e-15), k
            assert R.close(ys, yr, 1e-12, 1e-15), k
            continue
        row = log[k // E]
        assert row[0] == k
        # both candidates: the new iterate and the mean since the restart
        xa = np.mean(hist_x, axis=0)
        ya = np.mean(hist_y, axis=0)
        mc = R.kkt(S, *R.to_unscaled(S, xr, yr))["maxresid"]
        ma = R.kkt(S, *R.to_unscaled(S, xa, ya))["maxresid"]
        assert R.close(row[1], mc, 1e-9, 1e-14), (k, row[1], mc)
        assert R.close(row[2], ma, 1e-9, 1e-14), (k, row[2], ma)
        Kc = R.kkt_omega(S, xr, yr, omega)
        Ka = R.kkt_omega(S, xa, ya, omega)
        assert R.close(row[3], Kc, 1e-10, 1e-14), (k, row[3], Kc)
        assert R.close(row[4], Ka, 1e-10, 1e-14), (k, row[4], Ka)
        assert _margin_ok(Ka, Kc)
        cand = 1 if Ka < Kc else 0
        assert row[6] == cand, k
        K = Ka if cand else Kc
        xc, yc = (xa, ya) if cand else (xr, yr)
        t = k - last_k
        for thr in (beta[0] * K_last, beta[1] * K_last, K_prev):
            if np.isfinite(thr):
                assert _margin_ok(K, thr), k
        fired, reason = R.restart_test(K, K_last, K_prev, t, k, beta)
        assert bool(row[5]) == fired, (k, reason)
        if fired:
            dx = np.linalg.norm(xc - xl)
            dy = np.linalg.norm(yc - yl)
            if omega_rule == 0:
                omega = R.omega_smoothed(omega, dx, dy, 0.5)
            elif dx > 1e-10 and dy > 1e-10:
                e = np.log(omega * dx / dy)
                pid_int += e
                omega = float(np.exp(np.log(omega) - (pid[0] * e + pid[1] * pid_int
                                                      + pid[2] * (e - pid_eprev))))
                pid_eprev = e
            # the restart point is the candidate; the averages start afresh
            assert R.close(xs, xc, 1e-12, 1e-15) and R.close(ys, yc, 1e-12, 1e-15), k
            xl, yl = xs.copy(), ys.copy()
            hist_x, hist_y = [], []
            last_k = k
            K_last = R.kkt_omega(S, xs, ys, omega)
            K_prev = np.inf
            restarts.append((k, reason, cand))
        else:
            assert R.close(xs, xr, 1e-12, 1e-15) and R.close(ys, yr, 1e-12, 1e-15), k
            K_prev = K
        # the update is checked one restart at a time: continue from the
        # logged weight (the distances are sums over many recomputed
        # iterates, so their rounding differs from the oracle's by ~1e-13)
        assert R.close(row[7], omega, 1e-10), (k, row[7], omega)
        omega = row[7]
        records.append((k, mc, ma))
    return restarts, records


CASES = [
    # (generator, eval_every, iterations)
    (lambda: lpgen.planted_uniform(m=60, n=150, k=4, seed=5), 8, 640),
    (lambda: lpgen.planted_powerlaw(m=80, n=300, kmax=40, seed=6), 4, 600),
    (lambda: lpgen.multicommodity(nodes=40, arcs=150, commodities=2, seed=7), 8, 800),
]


def test_averaged_variant_replayed_from_its_definitions(oracle):
    reasons, cands = set(), set()
    for make, E, T in CASES:
        restarts, _ = replay_averaged(oracle, make(), E, T)
        assert restarts, "no restart to pin"
        reasons |= {r for _, r, _ in restarts}
        cands |= {c for _, _, c in restarts}
    # every branch of the rule has been exercised somewhere
    assert reasons == {1, 2, 3}, reasons
    assert cands == {0, 1}, cands


def test_averaged_variant_with_bounds_and_warm_start(oracle):
    lp = lpgen.planted_uniform(m=50, n=120, k=4, seed=8)
    rng = np.random.default_rng(8)
    l = -rng.uniform(0.0, 0.4, lp.n)
    x0 = np.maximum(l, rng.standard_normal(lp.n))
    y0 = rng.standard_normal(lp.m)
    restarts, _ = replay_averaged(oracle, lp, 8, 400, l=l, x0=x0, y0=y0)
    assert restarts


def test_pid_weight_replayed(oracle):
    # the PID controller's state (integral, previous error) carried across
    # restarts, with all three gains nonzero
    lp = lpgen.planted_powerlaw(m=80, n=300, kmax=40, seed=6)
    restarts, _ = replay_averaged(oracle, lp, 4, 600, omega_rule=1,
                                  pid=(0.7, 0.2, 0.1))
    assert len(restarts) >= 3


@pytest.mark.parametrize("beta", [(0.3, 0.7, 0.5), (0.1, 0.9, 0.2)])
def test_restart_thresholds_are_parameters(oracle, beta):
    # other thresholds: the replay with the same values must still agree
    lp = lpgen.planted_uniform(m=60, n=150, k=4, seed=5)
    restarts, _ = replay_averaged(oracle, lp, 8, 480, beta=beta)
    assert restarts


def test_snapshots_at_first_evaluation_reaching_recomputed_maxresid(oracle):
    # Algorithm 1's test on the better candidate, with maxresid recomputed
    # from the traced iterates (not read from the oracle's log)
    lp = lpgen.planted_uniform(m=30, n=80, k=3, seed=1)
    E, T = 8, 1400
    levels = oracle.alg1_levels(1e-1, 1e-6)
    _, records = replay_averaged(oracle, lp, E, T)
    r = oracle.solve(lp, levels=levels, eps_rel=1e-30, max_iters=T, eval_every=E)
    dr, dc, _ = oracle.ruiz(lp, 10)
    S = R.scaled(lp, dr, dc)
    m0 = R.kkt(S, np.zeros(lp.n), np.zeros(lp.m))["maxresid"]
    seq = [(0, m0)] + [(k, min(mc, ma)) for k, mc, ma in records]
    expect = []
    for lev in levels:
        hit = [k for k, mr in seq if mr <= lev]
        if not hit:
            break
        for _, mr in seq:
            assert _margin_ok(mr, lev)
        expect.append((lev, hit[0]))
    assert len(expect) == len(levels)
    assert [(s["level"], s["iter"]) for s in r.snaps] == expect


def replay_halpern(oracle, lp, E, T, rho=1.0, l=None):
    r = oracle.solve(lp, l=l, eps_rel=1e-30, max_iters=T, trace_k=T,
                     eval_every=E, variant=1, reflect=rho)
    assert r.info["status"] == 2 and r.info["iters"] == T
    dr, dc, _ = oracle.ruiz(lp, 10)
    S = R.scaled(lp, dr, dc, l)
    eta, omega = r.info["eta"], r.info["omega0"]
    log = r.eval_log
    X = r.trace_x / dc[None, :]
    Y = r.trace_y / dr[None, :]
    xs, ys = np.zeros(lp.n), np.zeros(lp.m)
    xa, ya = xs.copy(), ys.copy()
    t = 0
    r_last = r_prev = np.inf
    restarts = []
    for k in range(0, T + 1):
        tau, sigma = eta / omega, eta * omega
        if k % E == 0:
            row = log[k // E]
            assert row[0] == k
            xh, yh = R.pdhg_step(S, xs, ys, tau, sigma)
            mz = R.kkt(S, *R.to_unscaled(S, xs, ys))["maxresid"]
            mh = R.kkt(S, *R.to_unscaled(S, xh, yh))["maxresid"]
            assert R.close(row[1], mz, 1e-9, 1e-14), (k, row[1], mz)
            assert R.close(row[2], mh, 1e-9, 1e-14), (k, row[2], mh)
            fx = float((xs - xh) @ (xs - xh))
            fy = float((ys - yh) @ (ys - yh))
            r_cur = np.sqrt(omega * fx + fy / omega)
            assert R.close(row[3], r_cur, 1e-9, 1e-15), (k, row[3], r_cur)
            fired = False
            if k == 0:
                r_last = r_cur
            else:
                for thr in (0.2 * r_last, 0.8 * r_last, r_prev):
                    if np.isfinite(thr):
                        assert _margin_ok(r_cur, thr), k
                fired, reason = R.restart_test(r_cur, r_last, r_prev, t, k)
                if fired:
                    omega = R.omega_smoothed(omega, np.linalg.norm(xh - xa),
                                             np.linalg.norm(yh - ya))
                    xs, ys = xh, yh
                    xa, ya = xh.copy(), yh.copy()
                    t = 0
                    r_last = np.sqrt(omega * fx + fy / omega)
                    r_prev = np.inf
                    restarts.append((k, reason))
                else:
                    r_prev = r_cur
            assert bool(row[5]) == fired, k
            assert R.close(row[4], r_last, 1e-9, 1e-15), (k, row[4], r_last)
            assert R.close(row[7], omega, 1e-10), k
            omega = row[7]
            if k >= 1:
                assert R.close(X[k - 1], xs, 1e-12, 1e-15), k
                assert R.close(Y[k - 1], ys, 1e-12, 1e-15), k
        if k == T:
            break
        if k >= 1:
            xs, ys = X[k - 1], Y[k - 1]
        tau, sigma = eta / omega, eta * omega
        xn, yn = R.halpern_step(S, xs, ys, xa, ya, t, tau, sigma, rho)
        if (k + 1) % E:
            assert R.close(X[k], xn, 1e-12, 1e-15), k + 1
            assert R.close(Y[k], yn, 1e-12, 1e-15), k + 1
        xs, ys = xn, yn
        t += 1
    return restarts


def test_halpern_first_steps_dense(oracle):
    # three steps from the anchor 0 written out with lambda_t = (t+1)/(t+2):
    # z1 = 1/2 (2 T(z0) - z0) + 1/2 z0 = T(z0) for rho = 1, and so on
    lp = lpgen.planted_uniform(m=40, n=90, k=4, seed=3)
    dr, dc, _ = oracle.ruiz(lp, 10)
    S = R.scaled(lp, dr, dc)
    for rho in (1.0, 0.5):
        r = oracle.solve(lp, eps_rel=1e-30, max_iters=3, trace_k=3,
                         eval_every=50, variant=1, reflect=rho)
        eta, om = r.info["eta"], r.info["omega0"]
        tau, sigma = eta / om, eta * om
        z0x, z0y = np.zeros(lp.n), np.zeros(lp.m)
        xs, ys = z0x, z0y
        lams = []
        for t in range(3):
            lam = (t + 1.0) / (t + 2.0)
            lams.append(lam)
            Tx, Ty = R.pdhg_step(S, xs, ys, tau, sigma)
            xs = lam * ((1 + rho) * Tx - rho * xs) + (1 - lam) * z0x
            ys = lam * ((1 + rho) * Ty - rho * ys) + (1 - lam) * z0y
            assert R.close(r.trace_x[t] / dc, xs, 1e-13, 1e-16), (rho, t)
            assert R.close(r.trace_y[t] / dr, ys, 1e-13, 1e-16), (rho, t)
        assert lams == [0.5, 2 / 3, 0.75]


@pytest.mark.parametrize("rho", [1.0, 0.6])
def test_halpern_variant_replayed_from_its_definitions(oracle, rho):
    reasons = set()
    for make, E, T in CASES[:2]:
        restarts = replay_halpern(oracle, make(), E, T, rho=rho)
        assert restarts
        reasons |= {rr for _, rr in restarts}
    assert 3 in reasons and (1 in reasons or 2 in reasons), reasons
