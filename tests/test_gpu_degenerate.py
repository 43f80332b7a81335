"""Degenerate and tiny problems through the HIP path (C ABI), checked against
closed forms, brute-force vertex enumeration and the FP64 CPU oracle.

Shapes the large workloads never produce: a single constraint row (the dual
step's matrix has one row, the primal step's n rows of one entry), a
diagonal matrix, an all-empty row and an all-empty column, and LPs of a few
variables whose optimum is known exactly.
"""
import numpy as np
import pytest

from paper_2510_24429_amd import lpgen
from tests.bruteforce import lp_optimum

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    import torch
    assert torch.cuda.is_available()
    from paper_2510_24429_amd.solver import Solver as S
    return S


def _dense_lp(A, b, c, name="dense"):
    rows, cols = np.nonzero(A)
    return lpgen.from_coo(A.shape[0], A.shape[1], rows, cols, A[rows, cols],
                          b, c, name=name)


def _solve(Solver, lp, eps, **kw):
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=eps, **kw)
        st = s.solve()
        x, y, z = s.get_iterate()
        return st, s.info(), x, y


@pytest.mark.parametrize("variant", [0, 1])
def test_one_row_lp_closed_form(Solver, variant):
    # min c^T x s.t. a^T x = beta, x >= 0, a > 0: p* = beta * min_j c_j / a_j
    rng = np.random.default_rng(7)
    n = 9
    a = rng.uniform(0.5, 2.0, n)
    c = rng.uniform(1.0, 3.0, n)
    beta = 2.5
    lp = _dense_lp(a[None, :], np.array([beta]), c)
    st, inf, x, _ = _solve(Solver, lp, 1e-11, eval_every=8, variant=variant)
    pstar = beta * np.min(c / a)
    assert st == 1
    assert abs(inf["kkt"]["pobj"] - pstar) <= 1e-9 * (1 + pstar)
    j = int(np.argmin(c / a))
    assert abs(x[j] - beta / a[j]) <= 1e-7


@pytest.mark.parametrize("variant", [0, 1])
def test_identity_matrix_closed_form(Solver, variant):
    # A = I: the only feasible point is x = b; every column is basic, so y = c
    rng = np.random.default_rng(3)
    n = 12
    b = rng.uniform(0.1, 1.0, n)
    c = rng.standard_normal(n)
    lp = _dense_lp(np.eye(n), b, c)
    st, inf, x, y = _solve(Solver, lp, 1e-11, eval_every=4, variant=variant)
    assert st == 1
    assert np.max(np.abs(x - b)) <= 1e-9
    assert abs(inf["kkt"]["pobj"] - c @ b) <= 1e-9 * (1 + abs(c @ b))
    assert np.max(np.abs(y - c)) <= 1e-8


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("shape", [(2, 4), (3, 6), (4, 8)])
def test_tiny_lps_match_vertex_enumeration(Solver, seed, shape, variant):
    m, n = shape
    lp = lpgen.tiny_dense(m, n, seed=100 * m + seed)
    p, d, _, _ = lp_optimum(lp.dense(), lp.b, lp.c)
    st, inf, _, _ = _solve(Solver, lp, 1e-10, eval_every=16,
                           max_iters=2_000_000, variant=variant)
    assert st == 1
    assert abs(inf["kkt"]["pobj"] - p) <= 1e-8 * (1 + abs(p))
    assert abs(inf["kkt"]["dobj"] - d) <= 1e-8 * (1 + abs(d))


@pytest.mark.parametrize("variant", [0, 1])
def test_empty_row_and_column_match_oracle(Solver, oracle, variant):
    # row 0 of A has no entries (b_0 = 0, so it is satisfied by any x) and
    # column 0 has none (its cost c_0 > 0 keeps x_0 at 0): Ruiz leaves their
    # factors at 1, and both SpMVs meet a zero-length row
    base = lpgen.planted_uniform(m=60, n=120, k=4, seed=9)
    A = base.dense()
    A = np.vstack([np.zeros((1, A.shape[1])), A])
    A = np.hstack([np.zeros((A.shape[0], 1)), A])
    b = np.concatenate([[0.0], base.b])
    c = np.concatenate([[0.7], base.c])
    lp = _dense_lp(A, b, c, name="empty_row_col")
    assert lp.a_rp[1] == 0 and lp.at_rp[1] == 0
    ref = oracle.solve(lp, eps_rel=1e-9, eval_every=16, variant=variant)
    st, inf, x, _ = _solve(Solver, lp, 1e-9, eval_every=16, variant=variant)
    assert st == 1 and ref.info["status"] == 1
    assert inf["iters"] == ref.info["iters"]
    for key in ("rel_p", "rel_d", "rel_gap", "maxresid"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
    assert x[0] == 0.0
    pstar = base.c @ base.x_star
    assert abs(inf["kkt"]["pobj"] - pstar) <= 1e-7 * (1 + abs(pstar))


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("kind", ["infeasible", "unbounded"])
def test_lps_without_optimum_end_as_the_oracle(Solver, oracle, kind, variant):
    """An infeasible LP (x1 + x2 = -1) runs to its iteration limit with finite
    iterates; an unbounded one (min -x1, x1 = x2) grows until the iterates
    overflow and reports NUMERICAL, as the oracle does; the first 100
    iterates match the oracle's within 1e-10."""
    if kind == "infeasible":
        lp = lpgen.from_coo(1, 2, [0, 0], [0, 1], [1.0, 1.0], [-1.0], [1.0, 1.0])
    else:
        lp = lpgen.from_coo(1, 2, [0, 0], [0, 1], [1.0, -1.0], [0.0], [-1.0, 0.0])
    kw = dict(eps_rel=1e-8, eval_every=8, variant=variant)
    tr = oracle.solve(lp, trace_k=100, max_iters=100, **kw)
    ref = oracle.solve(lp, max_iters=20000, **kw)
    with Solver.from_lp(lp) as s:
        s.configure(**kw)
        for k in range(100):
            s.iterate(1)
            x, y, _ = s.get_iterate()
            scale_x = max(np.max(np.abs(tr.trace_x[k])), 1e-300)
            scale_y = max(np.max(np.abs(tr.trace_y[k])), 1e-300)
            assert np.max(np.abs(x - tr.trace_x[k])) <= 1e-10 * scale_x, k
            assert np.max(np.abs(y - tr.trace_y[k])) <= 1e-10 * scale_y, k
        s.configure(max_iters=20000, **kw)
        st = s.solve()
        inf = s.info()
    assert st == ref.info["status"] == (2 if kind == "infeasible" else 5)
    if kind == "infeasible":
        assert inf["iters"] == ref.info["iters"] == 20000
    else:
        # the evaluation at which a sum first overflows may differ by one
        assert abs(inf["iters"] - ref.info["iters"]) <= kw["eval_every"]


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("with_l", [False, True])
def test_matrix_without_nonzeros(Solver, oracle, variant, with_l):
    """A = 0 (3 x 4, no entries), b = 0, c > 0: no row block has work, the
    power iteration falls back to 1, and x = max(0, l) is optimal; status,
    iterations and x as the oracle's."""
    e = np.array([], dtype=np.int64)
    lp = lpgen.from_coo(3, 4, e, e, np.array([]), np.zeros(3),
                        np.array([1.0, 2.0, 0.5, 1.0]), name="zero")
    l = np.array([0.5, 0.0, 2.0, 1.0]) if with_l else None
    kw = dict(eps_rel=1e-10, max_iters=1000, variant=variant)
    ref = oracle.solve(lp, l=l, **kw)
    with Solver.from_lp(lp, lb=l) as s:
        s.configure(**kw)
        assert s.info()["sigma_hat"] == ref.info["sigma_hat"] == 1.0
        assert s.solve() == ref.info["status"] == 1
        assert s.info()["iters"] == ref.info["iters"]
        x, _, _ = s.get_iterate()
    assert np.array_equal(x, np.zeros(4) if l is None else l)
