"""Structure of the seeded synthetic inputs (the recipe the workloads state)."""
import numpy as np

from paper_2510_24429_amd import lpgen


def _check_pair(lp):
    assert lp.a_rp[0] == 0 and lp.a_rp[-1] == lp.nnz
    assert lp.at_rp[0] == 0 and lp.at_rp[-1] == lp.nnz
    rows = np.repeat(np.arange(lp.m), np.diff(lp.a_rp))
    # A^T is A's transpose, values bitwise
    perm = lp.a_perm_to_at()
    assert np.array_equal(lp.at_v[perm], lp.a_v)
    assert np.array_equal(lp.at_ci[perm], rows)
    # sorted, distinct column indices per row
    d = np.diff(lp.a_ci.astype(np.int64))
    starts = lp.a_rp[1:-1]
    ok = np.ones(lp.nnz - 1, dtype=bool)
    ok[starts[(starts > 0) & (starts < lp.nnz)] - 1] = False
    assert np.all(d[ok] > 0)


def test_uniform_small():
    lp = lpgen.make("uniform_m500_n1k")
    assert (lp.m, lp.n, lp.nnz) == (500, 1000, 5000)
    assert np.all(np.diff(lp.at_rp) == 5)
    _check_pair(lp)
    A = lp.dense()
    assert np.allclose(A @ lp.x_star, lp.b, atol=1e-13)
    assert np.allclose(A.T @ lp.y_star + lp.z_star, lp.c, atol=1e-13)
    assert lp.x_star @ lp.z_star == 0.0
    assert np.count_nonzero(lp.x_star) == 400
    assert np.all(lp.x_star >= 0) and np.all(lp.z_star >= 0)


def test_powerlaw_counts_and_bins():
    rng = np.random.default_rng(0)
    k = lpgen.powerlaw_counts(rng, 200_000, 2.1, 2, 5000)
    assert k.min() >= 2 and k.max() <= 5000
    assert abs(k.mean() - 9.49) < 0.6          # mean of the discrete law
    lp = lpgen.planted_powerlaw(m=20_000, n=100_000, seed=1)
    _check_pair(lp)
    L = np.diff(lp.at_rp)
    share = np.bincount(np.digitize(L, [9, 65, 1025]), weights=L) / L.sum()
    assert share[0] > 0.15 and share[3] > 0.02


def test_multicommodity_shape():
    lp = lpgen.multicommodity(nodes=1500, arcs=6000, commodities=8, seed=2)
    assert lp.m == 8 * 1500 + 1500 and lp.n == 8 * 6000 + 1500
    assert lp.nnz == 3 * 8 * 6000 + 1500
    _check_pair(lp)
    L = np.diff(lp.at_rp)
    assert set(np.unique(L)) == {1, 3}
    # supplies balance per commodity
    sup = lp.b[:8 * 1500].reshape(8, 1500).sum(axis=1)
    assert np.allclose(sup, 0.0, atol=1e-9)


def test_coupled_shape():
    lp = lpgen.planted_coupled(m=5000, n=20000, k=5, n_coupling=5,
                               coupling_len=2000, seed=4)
    assert lp.nnz == 5 * 20000 + 5 * 2000
    L = np.diff(lp.a_rp)
    assert np.all(L[-5:] == 2000)
    _check_pair(lp)
    A = lp.dense()
    assert np.allclose(A @ lp.x_star, lp.b, atol=1e-12)


def test_seeded_reproducible():
    a = lpgen.make("uniform_m500_n1k")
    b = lpgen.make("uniform_m500_n1k")
    assert np.array_equal(a.a_v, b.a_v) and np.array_equal(a.b, b.b)


def test_planted_flat_has_cost_in_the_row_space():
    lp = lpgen.planted_flat(200, 700, 5, 3)
    A = lp.dense()
    assert np.allclose(A @ lp.x_star, lp.b, rtol=1e-12, atol=1e-12)
    assert np.allclose(A.T @ lp.y_star, lp.c, rtol=1e-12, atol=1e-12)
    assert np.all(lp.x_star > 0)
