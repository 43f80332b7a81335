"""Pins of the FP64 CPU oracle against facts the paper and the mathematics fix.

None of these tests re-types the oracle's formulas: they compare it with
brute-force vertex enumeration, closed-form LPs, invariants that must hold
for any correct implementation, the planted optimum of the generators, and
the worked snapshot schedules printed in the paper.
"""
import os

import numpy as np
import pytest

from paper_2510_24429_amd import lpgen
from tests.bruteforce import lp_optimum

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense_lp(A, b, c, name="dense"):
    rows, cols = np.nonzero(A)
    return lpgen.from_coo(A.shape[0], A.shape[1], rows, cols, A[rows, cols],
                          b, c, name=name)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("shape", [(2, 4), (3, 6), (4, 8)])
def test_optimum_matches_vertex_enumeration(oracle, seed, shape, variant):
    m, n = shape
    lp = lpgen.tiny_dense(m, n, seed=100 * m + seed)
    A = lp.dense()
    p, d, pv, dv = lp_optimum(A, lp.b, lp.c)
    assert abs(p - d) <= 1e-9 * (1 + abs(p))          # strong duality
    r = oracle.solve(lp, eps_rel=1e-10, eval_every=16, max_iters=2_000_000,
                     variant=variant)
    assert r.info["status"] == 1
    assert abs(r.kkt["pobj"] - p) <= 1e-8 * (1 + abs(p))
    assert abs(r.kkt["dobj"] - d) <= 1e-8 * (1 + abs(d))
    # weak duality between every primal and dual vertex
    for x in pv:
        for y in dv:
            assert lp.b @ y <= lp.c @ x + 1e-9


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_planted_optimum_value(oracle, seed, variant):
    lp = lpgen.planted_uniform(m=60, n=120, k=4, seed=seed)
    pstar = lp.c @ lp.x_star
    assert abs(pstar - lp.b @ lp.y_star) <= 1e-10 * (1 + abs(pstar))
    r = oracle.solve(lp, eps_rel=1e-9, variant=variant)
    assert r.info["status"] == 1
    assert abs(r.kkt["pobj"] - pstar) <= 1e-7 * (1 + abs(pstar))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("variant", [0, 1])
def test_one_row_lp_closed_form(oracle, variant):
    # min c^T x s.t. a^T x = beta, x >= 0 with a > 0: p* = beta * min c_j / a_j
    rng = np.random.default_rng(7)
    n = 9
    a = rng.uniform(0.5, 2.0, n)
    c = rng.uniform(1.0, 3.0, n)
    beta = 2.5
    lp = _dense_lp(a[None, :], np.array([beta]), c)
    r = oracle.solve(lp, eps_rel=1e-11, eval_every=8, variant=variant)
    pstar = beta * np.min(c / a)
    assert r.info["status"] == 1
    assert abs(r.kkt["pobj"] - pstar) <= 1e-9 * (1 + pstar)
    j = int(np.argmin(c / a))
    assert abs(r.x[j] - beta / a[j]) <= 1e-7


@pytest.mark.parametrize("variant", [0, 1])
def test_identity_matrix_closed_form(oracle, variant):
    # A = I: the only feasible point is x = b, so p* = c^T b, y = c - z
    rng = np.random.default_rng(3)
    n = 12
    b = rng.uniform(0.1, 1.0, n)
    c = rng.standard_normal(n)
    lp = _dense_lp(np.eye(n), b, c)
    r = oracle.solve(lp, eps_rel=1e-11, eval_every=4, variant=variant)
    assert r.info["status"] == 1
    assert np.max(np.abs(r.x - b)) <= 1e-9
    assert abs(r.kkt["pobj"] - c @ b) <= 1e-9 * (1 + abs(c @ b))
    # every column is basic, so the dual is y = c, z = 0
    assert np.max(np.abs(r.y - c)) <= 1e-8


def test_kkt_at_planted_point_and_perturbations(oracle):
    lp = lpgen.planted_uniform(m=50, n=100, k=4, seed=11)
    A = lp.dense()
    k0 = oracle.kkt(lp, lp.x_star, lp.y_star, want_z=True)
    assert k0["maxresid"] <= 1e-14
    assert np.max(np.abs(k0["z"] - lp.z_star)) <= 1e-13
    # primal perturbation along e_j: ||r_P|| = delta * ||A[:, j]||
    j, delta = 17, 0.25
    x = lp.x_star.copy()
    x[j] += delta
    k1 = oracle.kkt(lp, x, lp.y_star)
    assert abs(k1["norm_rp"] - delta * np.linalg.norm(A[:, j])) <= 1e-13
    assert abs(k1["rp_inf"] - delta * np.max(np.abs(A[:, j]))) <= 1e-13
    assert k1["norm_rd"] <= 1e-13
    # gap: c^T x - b^T y = c^T x* + delta c_j - b^T y* = delta * c_j
    assert abs((k1["pobj"] - k1["dobj"]) - delta * lp.c[j]) <= 1e-12
    # dual perturbation along e_i by a large delta: r_D = max(0, delta a_i - z*)
    i, big = 5, 50.0
    y = lp.y_star.copy()
    y[i] += big
    k2 = oracle.kkt(lp, lp.x_star, y)
    expect = np.maximum(0.0, big * A[i, :] - lp.z_star)
    assert abs(k2["norm_rd"] - np.linalg.norm(expect)) <= 1e-11
    assert k2["norm_rp"] <= 1e-13
    assert abs(k2["rel_d"] - np.linalg.norm(expect) / (1 + np.linalg.norm(lp.c))) <= 1e-13


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("variant", [0, 1])
def test_iterates_respect_bounds_and_gap_identity(oracle, variant):
    lp = lpgen.planted_uniform(m=80, n=160, k=5, seed=2)
    rng = np.random.default_rng(2)
    l = -rng.uniform(0.0, 0.5, lp.n)
    r = oracle.solve(lp, l=l, eps_rel=1e-30, max_iters=150, trace_k=150,
                     eval_every=32, variant=variant)
    A = lp.dense()
    for k in range(150):
        x, y = r.trace_x[k], r.trace_y[k]
        # projection is exact in the scaled space; unscaling D_c (l / D_c)
        # may round l by an ulp.  (The Halpern iterate is a combination of
        # projected and unprojected points and is not bound to x >= l.)
        if variant == 0:
            assert np.all(x >= l - 4.5e-16 * np.abs(l))
        # c^T x - b^T y - l^T z = z^T (x - l) - r_D^T x - y^T r_P   (any x, y)
        d = lp.c - A.T @ y
        z = np.maximum(0.0, d)
        rD = A.T @ y + z - lp.c
        rP = lp.b - A @ x
        lhs = lp.c @ x - lp.b @ y - l @ z
        rhs = z @ (x - l) - rD @ x - y @ rP
        assert abs(lhs - rhs) <= 1e-11 * (1 + np.abs(lp.c) @ np.abs(x) + np.abs(lp.b) @ np.abs(y))
        assert np.all(z >= 0)


def test_bounded_lp_with_lower_bounds_matches_shift(oracle):
    # x >= l  is  x' = x - l >= 0 with b' = b - A l: same optimal x, objective
    # shifted by c^T l
    lp = lpgen.planted_uniform(m=40, n=90, k=4, seed=9)
    rng = np.random.default_rng(9)
    l = -rng.uniform(0.0, 0.3, lp.n)
    r1 = oracle.solve(lp, l=l, eps_rel=1e-10)
    A = lp.dense()
    lp2 = _dense_lp(A, lp.b - A @ l, lp.c)
    r2 = oracle.solve(lp2, eps_rel=1e-10)
    assert r1.info["status"] == 1 and r2.info["status"] == 1
    assert abs(r1.kkt["pobj"] - (r2.kkt["pobj"] + lp.c @ l)) <= 1e-7 * (1 + abs(r1.kkt["pobj"]))


# ---------------------------------------------------------------- Ruiz

def test_ruiz_bounds_and_convergence(oracle):
    lp = lpgen.planted_powerlaw(m=300, n=1500, kmax=200, seed=4)
    A = lp.dense()
    _, _, vs1 = oracle.ruiz(lp, 1)
    assert np.max(np.abs(vs1)) <= 1.0 + 4e-16            # |a|/sqrt(rho kappa) <= 1
    dr, dc, vs = oracle.ruiz(lp, 10)
    S = np.zeros_like(A)
    rows = np.repeat(np.arange(lp.m), np.diff(lp.a_rp))
    S[rows, lp.a_ci] = vs
    rmax = np.abs(S).max(axis=1)
    cmax = np.abs(S).max(axis=0)
    assert np.all(rmax <= 1 + 1e-15) and np.all(cmax <= 1 + 1e-15)
    assert np.all(rmax >= 1 - 2e-2) and np.all(cmax >= 1 - 2e-2)
    # l_inf Ruiz converges linearly: 40 passes equilibrate to ~1e-10
    _, _, vs40 = oracle.ruiz(lp, 40)
    S40 = np.zeros_like(A)
    S40[rows, lp.a_ci] = vs40
    assert np.all(np.abs(S40).max(axis=1) >= 1 - 1e-9)
    assert np.all(np.abs(S40).max(axis=0) >= 1 - 1e-9)
    # the scaled matrix is D_r A D_c
    assert np.allclose(S, dr[:, None] * A * dc[None, :], rtol=1e-15, atol=0)


def test_ruiz_diagonal_and_scale_invariance(oracle):
    d = np.array([4.0, 0.25, 16.0, 1.0])
    lp = _dense_lp(np.diag(d), np.ones(4), np.ones(4))
    dr, dc, vs = oracle.ruiz(lp, 1)
    # one pass on a diagonal matrix: D_r = D_c = 1/sqrt(|d|), scaled entries 1
    assert np.array_equal(dr, 1 / np.sqrt(d)) and np.array_equal(vs, np.ones(4))
    lp = lpgen.planted_uniform(m=30, n=70, k=3, seed=1)
    lp2 = lpgen.planted_uniform(m=30, n=70, k=3, seed=1)
    lp2.a_v = lp2.a_v * 4.0                           # power of 2: exact
    _, _, v1 = oracle.ruiz(lp, 10)
    _, _, v2 = oracle.ruiz(lp2, 10)
    assert np.array_equal(v1, v2)


# ---------------------------------------------------------------- power iteration

def test_power_iteration_vs_dense_norm(oracle):
    lp = lpgen.make("uniform_m500_n1k")
    _, _, vs = oracle.ruiz(lp, 10)
    S = np.zeros((lp.m, lp.n))
    rows = np.repeat(np.arange(lp.m), np.diff(lp.a_rp))
    S[rows, lp.a_ci] = vs
    exact = np.linalg.norm(S, 2)
    est = oracle.power(lp, vs, 100)
    assert est <= exact * (1 + 1e-12)
    assert est >= exact * 0.97
    est500 = oracle.power(lp, vs, 500)
    assert abs(est500 - exact) <= abs(est - exact) + 1e-12


# ---------------------------------------------------------------- schedule

def _golden_schedules():
    out = []
    with open(os.path.join(GOLDEN, "alg1_schedule.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split(":")
            ec, er = map(float, lhs.split())
            out.append((ec, er, [float(t) for t in rhs.split()]))
    return out


@pytest.mark.parametrize("ec,er,expect", _golden_schedules())
def test_alg1_levels_worked_examples(oracle, ec, er, expect):
    got = oracle.alg1_levels(ec, er)
    assert len(got) == len(expect)
    for g, e in zip(got, expect):
        assert abs(g - e) <= 1e-15 * e


def test_snapshots_fire_at_first_qualifying_evaluation(oracle):
    lp = lpgen.make("uniform_m500_n1k")
    levels = oracle.alg1_levels(1e-2, 1e-6)
    r = oracle.solve(lp, levels=levels, eps_rel=1e-6, keep_snap_vectors=True)
    assert r.info["status"] == 1
    assert [s["level"] for s in r.snaps] == levels
    log = r.eval_log
    assert log[0, 0] == 0 and np.isnan(log[0, 2])     # the k = 0 check
    best = np.fmin(log[:, 1], log[:, 2])
    for i, s in enumerate(r.snaps):
        assert s["maxresid"] <= s["level"]
        # first evaluation at which the better candidate reached the level
        first = log[best <= s["level"], 0]
        k0 = 0 if s["iter"] == 0 else int(first[0])
        assert s["iter"] == k0
        # the stored snapshot is the iterate it claims: recompute its KKT
        kk = oracle.kkt(lp, r.snap_x[i], r.snap_y[i], want_z=True)
        assert abs(kk["maxresid"] - s["maxresid"]) <= 1e-12
        assert np.array_equal(kk["z"], r.snap_z[i])
    # literal Algorithm 1: at most one level per check
    rl = oracle.solve(lp, levels=levels, eps_rel=1e-6, literal_snapshots=1)
    its = [s["iter"] for s in rl.snaps]
    assert len(set(its)) == len(its)
    assert [s["level"] for s in rl.snaps] == levels


def test_terminates_on_best_candidate(oracle):
    lp = lpgen.make("uniform_m500_n1k")
    r = oracle.solve(lp, eps_rel=1e-6)
    kk = oracle.kkt(lp, r.x, r.y)
    assert kk["maxresid"] <= 1e-6
    assert abs(kk["maxresid"] - r.kkt["maxresid"]) <= 1e-15
    assert r.info["iters"] % 64 == 0


def test_status_codes(oracle):
    lp = lpgen.make("uniform_m500_n1k")
    r = oracle.solve(lp, eps_rel=1e-12, max_iters=100)
    assert r.info["status"] == 2 and r.info["iters"] == 100
    b = lp.b.copy()
    b[3] = np.nan
    r = oracle.solve(lp, b=b, eps_rel=1e-6, max_iters=1000)
    assert r.info["status"] == 5
    # starting at the planted optimum terminates at k = 0 and emits every level
    r = oracle.solve(lp, x0=lp.x_star, y0=lp.y_star, levels=[1e-4, 1e-6],
                     eps_rel=1e-6)
    assert r.info["status"] == 1 and r.info["iters"] == 0
    assert [s["iter"] for s in r.snaps] == [0, 0]


# ---------------------------------------------------------------- refinement

def test_fp64_refinement_reaches_1e8(oracle):
    lp = lpgen.make("uniform_m500_n1k")
    out = oracle.refine(lp, outer_eps=1e-8, max_rounds=6, eps_rel=1e-4)
    assert out["status"] == 1
    kk = oracle.kkt(lp, out["x"], out["y"])
    assert kk["maxresid"] <= 1e-8
    pstar = lp.c @ lp.x_star
    assert abs(kk["pobj"] - pstar) <= 1e-8 * (1 + abs(pstar))
    assert np.all(out["x"] >= 0)


# ---------------------------------------------------------------- adjoint

def _fd_check(oracle, lp, dr, dc, tau, sigma, K, xt, g, which, idx, h=1e-6):
    base, h0 = oracle.unrolled_fwd(lp, dr, dc, tau, sigma, K)
    errs = []
    for t in idx:
        args_p, args_m = {}, {}
        if which == "c":
            vp, vm = lp.c.copy(), lp.c.copy()
            key = "c"
        elif which == "b":
            vp, vm = lp.b.copy(), lp.b.copy()
            key = "b"
        else:
            vp, vm = lp.a_v.copy(), lp.a_v.copy()
            key = "vals"
        vp[t] += h
        vm[t] -= h
        xp, hp = oracle.unrolled_fwd(lp, dr, dc, tau, sigma, K, **{key: vp})
        xm, hm = oracle.unrolled_fwd(lp, dr, dc, tau, sigma, K, **{key: vm})
        if hp != h0 or hm != h0:
            continue                              # at a kink: skip
        fd = np.sum((xp - xm) * (xp + xm - 2 * xt)) / (2 * h)
        errs.append(abs(fd - g[t]) / max(abs(g[t]), 1e-3 * np.max(np.abs(g))))
    return errs


def test_adjoint_vs_central_differences(oracle):
    lp = lpgen.planted_uniform(m=60, n=120, k=4, seed=5)
    dr, dc, vs = oracle.ruiz(lp, 10)
    eta = 0.9 / oracle.power(lp, vs)
    xt = lpgen.target_vector(lp.n, 5)
    K = 40
    _, L, gc, gb, gA = oracle.unrolled(lp, dr, dc, eta, eta, K, xt)
    rng = np.random.default_rng(1)
    for which, g, size in (("c", gc, lp.n), ("b", gb, lp.m), ("A", gA, lp.nnz)):
        errs = _fd_check(oracle, lp, dr, dc, eta, eta, K, xt, g, which,
                         rng.choice(size, 12, replace=False))
        assert len(errs) >= 6
        assert max(errs) <= 1e-6, (which, errs)


def test_adjoint_one_step_closed_form(oracle):
    # K = 1 from zero: x_1 = D_c max(0, -tau c~), so
    # dL/dc_j = 2 (x_1j - t_j) * D_c,j * (-tau) * D_c,j * 1[-tau c~_j > 0]
    lp = lpgen.planted_uniform(m=20, n=50, k=3, seed=8)
    dr, dc, _ = oracle.ruiz(lp, 10)
    xt = lpgen.target_vector(lp.n, 8)
    tau, sigma = 0.3, 0.2
    xK, L, gc, gb, gA = oracle.unrolled(lp, dr, dc, tau, sigma, 1, xt)
    cs = dc * lp.c
    x1 = dc * np.maximum(0.0, -tau * cs)
    assert np.allclose(xK, x1, rtol=0, atol=1e-15)
    expect = 2 * (x1 - xt) * dc * (-tau) * dc * (-tau * cs > 0)
    assert np.allclose(gc, expect, rtol=1e-14, atol=1e-15)
    # y_1 = sigma (b~ - A~ (2 x_1)) never reaches the loss in one step
    assert np.all(gb == 0.0)
    assert abs(L - np.sum((x1 - xt) ** 2)) <= 1e-12


def test_adjoint_linearity_transpose(oracle):
    # with masks frozen the K-step map is affine in (c, b); the reverse pass is
    # its transpose: <J u, w> = <u, J^T w> checked through a directional
    # difference (exact for an affine map, up to rounding)
    lp = lpgen.planted_uniform(m=40, n=80, k=4, seed=6)
    dr, dc, vs = oracle.ruiz(lp, 10)
    eta = 0.9 / oracle.power(lp, vs)
    K = 25
    xt = lpgen.target_vector(lp.n, 6)
    x0, h0 = oracle.unrolled_fwd(lp, dr, dc, eta, eta, K)
    rng = np.random.default_rng(0)
    w = rng.standard_normal(lp.n)
    # loss whose gradient at x_K is w:  L = ||x_K - xt||^2 with xt = x_K - w/2
    xt = x0 - 0.5 * w
    _, _, gc, gb, _ = oracle.unrolled(lp, dr, dc, eta, eta, K, xt)
    for _ in range(3):
        uc = rng.standard_normal(lp.n)
        ub = rng.standard_normal(lp.m)
        h = 1e-7
        xp, hp = oracle.unrolled_fwd(lp, dr, dc, eta, eta, K, c=lp.c + h * uc, b=lp.b + h * ub)
        if hp != h0:
            continue
        jvp = (xp - x0) / h
        lhs = w @ jvp
        rhs = uc @ gc + ub @ gb
        assert abs(lhs - rhs) <= 1e-6 * (abs(lhs) + abs(rhs) + 1e-12)


def test_halpern_first_step_is_the_pdhg_step(oracle):
    # with reflection rho = 1 and lambda = 1/2 the first Halpern step from the
    # anchor z0 gives z1 = (1/2)(2 T(z0) - z0) + (1/2) z0 = T(z0), i.e. the
    # averaged variant's first iterate; rho = 0 gives the midpoint of z0 = 0
    # and T(z0)
    lp = lpgen.planted_uniform(m=40, n=90, k=4, seed=3)
    a = oracle.solve(lp, eps_rel=1e-30, max_iters=1, trace_k=1, eval_every=50)
    h = oracle.solve(lp, eps_rel=1e-30, max_iters=1, trace_k=1, eval_every=50,
                     variant=1)
    assert np.allclose(h.trace_x[0], a.trace_x[0], rtol=0, atol=1e-15)
    assert np.allclose(h.trace_y[0], a.trace_y[0], rtol=0, atol=1e-15)
    h0 = oracle.solve(lp, eps_rel=1e-30, max_iters=1, trace_k=1, eval_every=50,
                      variant=1, reflect=0.0)
    assert np.allclose(h0.trace_x[0], 0.5 * a.trace_x[0], rtol=0, atol=1e-15)


def test_halpern_needs_fewer_iterations(oracle):
    lp = lpgen.make("uniform_m500_n1k")
    a = oracle.solve(lp, eps_rel=1e-8)
    h = oracle.solve(lp, eps_rel=1e-8, variant=1)
    assert a.info["status"] == h.info["status"] == 1
    assert h.info["iters"] < a.info["iters"]
    pstar = lp.c @ lp.x_star
    assert abs(h.kkt["pobj"] - pstar) <= 1e-7 * (1 + abs(pstar))


def test_halpern_returns_projected_point(oracle):
    lp = lpgen.planted_uniform(m=80, n=160, k=5, seed=2)
    rng = np.random.default_rng(2)
    l = -rng.uniform(0.0, 0.5, lp.n)
    r = oracle.solve(lp, l=l, eps_rel=1e-8, variant=1,
                     levels=[1e-3, 1e-5, 1e-8], keep_snap_vectors=True)
    assert r.info["status"] == 1
    assert np.all(r.x >= l - 4.5e-16 * np.abs(l))
    for i in range(len(r.snaps)):
        assert np.all(r.snap_x[i] >= l - 4.5e-16 * np.abs(l))


@pytest.mark.parametrize("variant", [0, 1])
def test_pid_with_proportional_gain_theta_is_the_smoothed_rule(oracle, variant):
    # log w - theta log(w dx / dy) = (1 - theta) log w + theta log(dy / dx):
    # the PID rule with kp = theta and no integral or derivative term is the
    # smoothed rule, up to the rounding of the two log forms
    lp = lpgen.planted_powerlaw(m=600, n=3000, kmax=300, seed=9)
    a = oracle.solve(lp, eps_rel=1e-8, variant=variant, omega_rule=0, omega_theta=0.5)
    b = oracle.solve(lp, eps_rel=1e-8, variant=variant, omega_rule=1, pid_kp=0.5,
                     pid_ki=0.0, pid_kd=0.0)
    assert a.info["status"] == b.info["status"] == 1
    assert a.info["restarts"] == b.info["restarts"]
    assert abs(a.info["iters"] - b.info["iters"]) <= 64
    assert abs(np.log(a.info["omega"]) - np.log(b.info["omega"])) <= 1e-6


def test_pid_rule_reaches_the_same_optimum(oracle):
    lp = lpgen.multicommodity(nodes=300, arcs=1200, commodities=3, seed=4)
    r0 = oracle.solve(lp, eps_rel=1e-8, variant=1)
    r1 = oracle.solve(lp, eps_rel=1e-8, variant=1, omega_rule=1)
    assert r0.info["status"] == r1.info["status"] == 1
    # each objective is within its weak-duality bound of the optimum p*:
    # pobj - p* <= (pobj - dobj) + ||r_D|| ||x*||, p* - pobj <= ||y*|| ||r_P||
    # (each run's own point stands in for x*, y*, with 10% slack)
    def bound(r, o):
        k = r.kkt
        nx = 1.1 * max(np.linalg.norm(r.x), np.linalg.norm(o.x))
        ny = 1.1 * max(np.linalg.norm(r.y), np.linalg.norm(o.y))
        return abs(k["pobj"] - k["dobj"]) + k["norm_rd"] * nx + k["norm_rp"] * ny
    assert abs(r0.kkt["pobj"] - r1.kkt["pobj"]) <= bound(r0, r1) + bound(r1, r0)


# ---------------------------------------------------------- polishing

@pytest.mark.parametrize("mode", [1, 2])
def test_feasibility_stop_measures(oracle, mode):
    # stop_on = 1 (2) stops on rel_p (rel_d) alone: the returned point meets
    # that measure, recomputed, and stops no later than the full test
    lp = lpgen.make("uniform_m500_n1k")
    full = oracle.solve(lp, eps_rel=1e-6)
    r = oracle.solve(lp, eps_rel=1e-6, stop_on=mode)
    k = oracle.kkt(lp, r.x, r.y)
    assert r.info["status"] == 1
    assert (k["rel_p"] if mode == 1 else k["rel_d"]) <= 1e-6
    assert r.info["iters"] <= full.info["iters"]


@pytest.mark.parametrize("variant", [0, 1])
def test_polishing_never_alters_the_main_iteration(oracle, variant):
    # on an LP where no polishing attempt succeeds, the solve with polishing
    # is the solve without it: same iterations, restarts, point and KKT
    lp = lpgen.planted_powerlaw(m=1500, n=6000, kmax=600, seed=3)
    a = oracle.solve(lp, eps_rel=1e-6, variant=variant)
    b = oracle.solve(lp, eps_rel=1e-6, variant=variant, polish=1)
    assert b.info["polish_attempts"] >= 1 and b.info["candidate"] != 2
    assert a.info["iters"] == b.info["iters"]
    assert a.info["restarts"] == b.info["restarts"]
    assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)
    assert a.kkt == b.kkt


def test_polishing_succeeds_when_feasibility_is_free(oracle):
    lp = lpgen.planted_flat(300, 1000, 5, 1)
    a = oracle.solve(lp, eps_rel=1e-8, variant=0)
    b = oracle.solve(lp, eps_rel=1e-8, variant=0, polish=1)
    assert b.info["status"] == 1 and b.info["candidate"] == 2
    assert b.info["iters"] < a.info["iters"]
    k = oracle.kkt(lp, b.x, b.y)
    assert k["maxresid"] <= 1e-8
    assert abs(k["maxresid"] - b.kkt["maxresid"]) <= 1e-12
    assert np.all(b.x >= 0)
