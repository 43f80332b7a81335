"""The CPU PDHG (the paper's CPU platform, Section 4.1) against the FP64
oracle: Ruiz factors bitwise, step size and primal weight, iterates over the
first 100 iterations element-wise within 1e-10, full solves with the same
iteration counts, restarts and snapshot points and final KKT within 1e-12,
in both variants; results independent of the thread count; status codes and
argument errors.  No GPU."""
import threading
import time

import numpy as np
import pytest

from paper_2510_24429_amd import lpgen
from paper_2510_24429_amd._lib import PDHGError
from paper_2510_24429_amd.cpu import CpuSolver, stream_bandwidth


def err(a, b):
    nb = np.linalg.norm(b)
    e1 = np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
    s = np.max(np.abs(b)) if b.size else 0.0
    e2 = np.max(np.abs(a - b)) / (s if s > 0 else 1.0) if a.size else 0.0
    return max(e1, e2)


def _trace(oracle, lp, K, threads=3, l=None, **kw):
    # the oracle stops at K: its traced window ends there
    ref = oracle.solve(lp, l=l, trace_k=K, max_iters=K, **kw)
    worst = 0.0
    with CpuSolver.from_lp(lp, lb=l, threads=threads) as s:
        s.configure(**kw)
        for k in range(K):
            s.iterate(1)
            x, y, _ = s.get_iterate()
            worst = max(worst, err(x, ref.trace_x[k]), err(y, ref.trace_y[k]))
    return worst


def test_scaling_and_step_size_match_oracle(oracle):
    for lp in (lpgen.make("uniform_m500_n1k"),
               lpgen.planted_powerlaw(m=2000, n=10000, kmax=1500, seed=7)):
        dr, dc, _ = oracle.ruiz(lp, 10)
        ref = oracle.solve(lp, eps_rel=1e-6, max_iters=0)
        with CpuSolver.from_lp(lp, threads=4) as s:
            s.configure(eps_rel=1e-6)
            gdr, gdc = s.get_scaling()
            inf = s.info()
        assert np.array_equal(gdr, dr) and np.array_equal(gdc, dc)
        for key in ("sigma_hat", "omega0", "eta"):
            assert abs(inf[key] - ref.info[key]) <= 1e-13 * abs(ref.info[key]), key


@pytest.mark.parametrize("variant", [0, 1])
def test_iterates_first_100_match_oracle(oracle, variant):
    lp = lpgen.make("uniform_m500_n1k")
    assert _trace(oracle, lp, 100, eps_rel=1e-8, variant=variant) <= 1e-10


@pytest.mark.parametrize("variant", [0, 1])
def test_iterates_match_with_lower_bounds_and_skew(oracle, variant):
    lp = lpgen.planted_powerlaw(m=3000, n=20000, kmax=2500, seed=21)
    l = -np.random.default_rng(12).uniform(0.0, 0.5, lp.n)
    w = _trace(oracle, lp, 100, threads=5, l=l, eps_rel=1e-8, eval_every=16,
               variant=variant)
    assert w <= 1e-10


def test_iterates_match_with_eval_every_iteration(oracle):
    lp = lpgen.make("uniform_m500_n1k")
    assert _trace(oracle, lp, 60, eps_rel=1e-8, eval_every=1) <= 1e-10


@pytest.mark.parametrize("variant,rule", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_full_solve_matches_oracle(oracle, variant, rule):
    lp = lpgen.make("uniform_m500_n1k")
    levels = [1e-2, 1e-4, 1e-6]
    kw = dict(eps_rel=1e-6, variant=variant, omega_rule=rule, eval_every=32)
    ref = oracle.solve(lp, levels=levels, keep_snap_vectors=True, **kw)
    with CpuSolver.from_lp(lp, threads=4) as s:
        s.configure(levels=levels, **kw)
        st = s.solve()
        inf = s.info()
        log = s.eval_log()
        snaps = [s.snapshot(i) for i in range(s.snapshot_count())]
        x, y, _ = s.get_iterate()
    assert st == 1 and ref.info["status"] == 1
    assert inf["iters"] == ref.info["iters"] and inf["restarts"] == ref.info["restarts"]
    assert inf["candidate"] == ref.info["candidate"]
    assert np.array_equal(log[:, 0], ref.eval_log[:, 0])
    assert np.array_equal(log[:, 5], ref.eval_log[:, 5])
    assert np.allclose(log[:, 7], ref.eval_log[:, 7], rtol=1e-10, atol=0)
    for key in ("rel_p", "rel_d", "rel_gap", "maxresid"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
    assert err(x, ref.x) <= 1e-9 and err(y, ref.y) <= 1e-9
    assert len(snaps) == len(ref.snaps) == 3
    for (info, sx, sy, sz), sn, rx, ry in zip(snaps, ref.snaps, ref.snap_x, ref.snap_y):
        assert info["level"] == sn["level"] and info["iter"] == sn["iter"]
        assert abs(info["maxresid"] - sn["maxresid"]) <= 1e-12
        assert err(sx, rx) <= 1e-9 and err(sy, ry) <= 1e-9
        assert oracle.kkt(lp, sx, sy)["maxresid"] <= sn["level"]
        assert np.all(sz >= 0)


def test_multicommodity_solve_matches_oracle(oracle):
    """The flow LP's dual is not unique (each commodity's conservation rows
    sum to zero), so over thousands of iterations y drifts along that
    direction by rounding (~1e-12 relative here) while the decisions stay the
    same.  The objectives are then compared through the bound the drift puts
    on them, |c^T dx| <= ||c|| ||dx|| and |b^T dy| <= ||b|| ||dy||."""
    lp = lpgen.multicommodity(nodes=300, arcs=1200, commodities=4, seed=5)
    kw = dict(eps_rel=1e-6, variant=1)
    ref = oracle.solve(lp, **kw)
    with CpuSolver.from_lp(lp, threads=3) as s:
        s.configure(**kw)
        assert s.solve() == 1
        inf = s.info()
        x, y, _ = s.get_iterate()
    assert inf["iters"] == ref.info["iters"] and inf["restarts"] == ref.info["restarts"]
    for key in ("rel_p", "rel_d"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
    assert err(x, ref.x) <= 1e-12 and err(y, ref.y) <= 1e-10
    tiny = 1e-12 * (1 + abs(ref.kkt["pobj"]))
    assert abs(inf["kkt"]["pobj"] - ref.kkt["pobj"]) <= \
        np.linalg.norm(lp.c) * np.linalg.norm(x - ref.x) + tiny
    assert abs(inf["kkt"]["dobj"] - ref.kkt["dobj"]) <= \
        np.linalg.norm(lp.b) * np.linalg.norm(y - ref.y) + tiny


def test_results_do_not_depend_on_thread_count():
    lp = lpgen.planted_powerlaw(m=3000, n=20000, kmax=2500, seed=22)
    out = []
    for T in (1, 3, 8):
        with CpuSolver.from_lp(lp, threads=T) as s:
            s.configure(eps_rel=1e-9, eval_every=16, variant=0)
            s.iterate(400)
            out.append((s.get_iterate(), s.eval_log(), s.info()))
    for (it, log, inf) in out[1:]:
        for a, b in zip(it, out[0][0]):
            assert np.array_equal(a, b)
        assert np.array_equal(log, out[0][1], equal_nan=True)
        assert inf["iters"] == out[0][2]["iters"]
    # a thread-pool change keeps the iterate and the course of the solve
    with CpuSolver.from_lp(lp, threads=2) as s:
        s.configure(eps_rel=1e-9, eval_every=16, variant=0)
        s.iterate(200)
        s.set_threads(6)
        s.iterate(200)
        for a, b in zip(s.get_iterate(), out[0][0]):
            assert np.array_equal(a, b)


def test_status_codes(oracle):
    lp = lpgen.make("uniform_m500_n1k")
    with CpuSolver.from_lp(lp, threads=2) as s:
        s.configure(eps_rel=1e-12, max_iters=100)
        assert s.solve() == 2                       # ITER_LIMIT
        assert s.info()["iters"] == 100
        s.configure(eps_rel=1e-14, time_limit_s=0.05, eval_every=8)
        assert s.solve() == 3                       # TIME_LIMIT
    b = lp.b.copy()
    b[3] = np.nan
    with CpuSolver(lp.m, lp.n, lp.a_rp, lp.a_ci, lp.a_v, lp.at_rp, lp.at_ci,
                   lp.at_v, b, lp.c) as s:
        s.configure(eps_rel=1e-6)
        assert s.solve() == 5                       # NUMERICAL
    big = lpgen.planted_powerlaw(m=4000, n=20000, kmax=1000, seed=3)
    with CpuSolver.from_lp(big, threads=2) as s:
        s.configure(eps_rel=1e-14, eval_every=8)
        threading.Timer(0.2, s.cancel).start()
        t0 = time.time()
        assert s.solve() == 4                       # CANCELLED
        assert time.time() - t0 < 30


def test_argument_errors():
    lp = lpgen.make("uniform_m500_n1k")
    at_v = lp.at_v.copy()
    at_v[0] += 1.0
    with pytest.raises(PDHGError, match="TRANSPOSE"):
        CpuSolver(lp.m, lp.n, lp.a_rp, lp.a_ci, lp.a_v, lp.at_rp, lp.at_ci, at_v,
                  lp.b, lp.c)
    with CpuSolver.from_lp(lp) as s:
        with pytest.raises(PDHGError, match="STATE"):
            s.iterate(1)
        with pytest.raises(PDHGError, match="FP64"):
            s.configure(precision=1)
        with pytest.raises(PDHGError, match="polishing"):
            s.configure(polish=1)
        with pytest.raises(PDHGError, match="descending"):
            s.configure(levels=[1e-6, 1e-4])


def test_stream_bandwidth_is_measured():
    g1 = stream_bandwidth(1, 1 << 26, 2)
    g2 = stream_bandwidth(2, 1 << 26, 2)
    assert g1 > 0.1 and g2 > 0.1


# ------------------------------------------------------- degenerate inputs
# The shapes of the GPU path's degenerate tests: one constraint row, A = I,
# tiny LPs whose optimum vertex enumeration finds, an empty row and column.

def _cpu_solve(lp, eps, threads=2, **kw):
    with CpuSolver.from_lp(lp, threads=threads) as s:
        s.configure(eps_rel=eps, **kw)
        st = s.solve()
        x, y, _ = s.get_iterate()
        return st, s.info(), x, y


def _from_dense(A, b, c, name="dense"):
    rows, cols = np.nonzero(A)
    return lpgen.from_coo(A.shape[0], A.shape[1], rows, cols, A[rows, cols], b, c,
                          name=name)


@pytest.mark.parametrize("variant", [0, 1])
def test_one_row_lp_closed_form(variant):
    # min c^T x s.t. a^T x = beta, x >= 0, a > 0: p* = beta * min_j c_j / a_j
    rng = np.random.default_rng(7)
    a = rng.uniform(0.5, 2.0, 9)
    c = rng.uniform(1.0, 3.0, 9)
    lp = _from_dense(a[None, :], np.array([2.5]), c)
    st, inf, x, _ = _cpu_solve(lp, 1e-11, eval_every=8, variant=variant)
    assert st == 1
    pstar = 2.5 * np.min(c / a)
    assert abs(inf["kkt"]["pobj"] - pstar) <= 1e-9 * (1 + pstar)
    j = int(np.argmin(c / a))
    assert abs(x[j] - 2.5 / a[j]) <= 1e-7


@pytest.mark.parametrize("variant", [0, 1])
def test_identity_matrix_closed_form(variant):
    # A = I: x = b is the only feasible point and y = c
    rng = np.random.default_rng(3)
    b = rng.uniform(0.1, 1.0, 12)
    c = rng.standard_normal(12)
    lp = _from_dense(np.eye(12), b, c)
    st, inf, x, y = _cpu_solve(lp, 1e-11, eval_every=4, variant=variant)
    assert st == 1
    assert np.max(np.abs(x - b)) <= 1e-9 and np.max(np.abs(y - c)) <= 1e-8


@pytest.mark.parametrize("seed,shape", [(0, (2, 4)), (1, (3, 6)), (2, (4, 8))])
def test_tiny_lps_match_vertex_enumeration(seed, shape):
    from tests.bruteforce import lp_optimum
    m, n = shape
    lp = lpgen.tiny_dense(m, n, seed=100 * m + seed)
    p, d, _, _ = lp_optimum(lp.dense(), lp.b, lp.c)
    st, inf, _, _ = _cpu_solve(lp, 1e-10, threads=1, eval_every=16,
                               max_iters=2_000_000, variant=1)
    assert st == 1
    assert abs(inf["kkt"]["pobj"] - p) <= 1e-8 * (1 + abs(p))
    assert abs(inf["kkt"]["dobj"] - d) <= 1e-8 * (1 + abs(d))


@pytest.mark.parametrize("variant", [0, 1])
def test_empty_row_and_column_match_oracle(oracle, variant):
    base = lpgen.planted_uniform(m=60, n=120, k=4, seed=9)
    A = base.dense()
    A = np.vstack([np.zeros((1, A.shape[1])), A])
    A = np.hstack([np.zeros((A.shape[0], 1)), A])
    lp = _from_dense(A, np.concatenate([[0.0], base.b]), np.concatenate([[0.7], base.c]))
    assert lp.a_rp[1] == 0 and lp.at_rp[1] == 0
    ref = oracle.solve(lp, eps_rel=1e-9, eval_every=16, variant=variant)
    st, inf, x, _ = _cpu_solve(lp, 1e-9, threads=3, eval_every=16, variant=variant)
    assert st == 1 and ref.info["status"] == 1
    assert inf["iters"] == ref.info["iters"]
    for key in ("rel_p", "rel_d", "rel_gap", "maxresid"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
    assert x[0] == 0.0


# ------------------------------------------------ LPs without an optimum
# An infeasible LP (x1 + x2 = -1, x >= 0) drives y along its infeasibility
# ray: the solve runs to its iteration limit with finite iterates.  An
# unbounded LP (min -x1, x1 - x2 = 0, x >= 0) drives x along its ray, and the
# primal-weight updates at restarts make the growth geometric until the
# iterates overflow: the solve reports NUMERICAL.  There is no infeasibility
# detection; both end as the oracle's do.

NO_OPTIMUM = {
    "infeasible": lambda: lpgen.from_coo(1, 2, [0, 0], [0, 1], [1.0, 1.0], [-1.0],
                                         [1.0, 1.0], name="infeasible"),
    "unbounded": lambda: lpgen.from_coo(1, 2, [0, 0], [0, 1], [1.0, -1.0], [0.0],
                                        [-1.0, 0.0], name="unbounded"),
}


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("kind", ["infeasible", "unbounded"])
def test_lps_without_optimum_end_as_the_oracle(oracle, kind, variant):
    lp = NO_OPTIMUM[kind]()
    kw = dict(eps_rel=1e-8, eval_every=8, variant=variant)
    assert _trace(oracle, lp, 100, threads=1, **kw) <= 1e-10
    ref = oracle.solve(lp, max_iters=20000, **kw)
    with CpuSolver.from_lp(lp, threads=1) as s:
        s.configure(max_iters=20000, **kw)
        st = s.solve()
        assert st == ref.info["status"] == (2 if kind == "infeasible" else 5)
        assert s.info()["iters"] == ref.info["iters"]
        x, y, _ = s.get_iterate()
        if kind == "infeasible":
            assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("with_l", [False, True])
def test_matrix_without_nonzeros(oracle, variant, with_l):
    """A = 0 (3 x 4, no entries), b = 0, c > 0: the power iteration finds no
    norm and falls back to 1; x = max(0, l) is optimal.  Status, iterations
    and x as the oracle's."""
    e = np.array([], dtype=np.int64)
    lp = lpgen.from_coo(3, 4, e, e, np.array([]), np.zeros(3),
                        np.array([1.0, 2.0, 0.5, 1.0]), name="zero")
    l = np.array([0.5, 0.0, 2.0, 1.0]) if with_l else None
    kw = dict(eps_rel=1e-10, max_iters=1000, variant=variant)
    ref = oracle.solve(lp, l=l, **kw)
    with CpuSolver.from_lp(lp, lb=l, threads=2) as s:
        s.configure(**kw)
        assert s.info()["sigma_hat"] == ref.info["sigma_hat"] == 1.0
        assert s.solve() == ref.info["status"] == 1
        assert s.info()["iters"] == ref.info["iters"]
        x, _, _ = s.get_iterate()
    assert np.array_equal(x, np.zeros(4) if l is None else l)
