"""Seeded synthetic standard-form LP generators (min c^T x, Ax = b, x >= 0).

This module only builds problem data: sparsity patterns, values, and the
right-hand sides of a planted primal-dual optimum.  It holds none of the
solver's arithmetic (no scaling, no PDHG step, no residual), so both the HIP
path and the CPU oracle can take their inputs from it without sharing code.

Every generator returns an ``LP`` with CSR A and an explicit CSR A^T built
from the same coordinate list, so A^T's values are bitwise A's values.
Index types: row pointers int64, column indices int32, values float64.

Problem families (sizes are the defaults; every one can be scaled down):

* ``planted_uniform``: k distinct uniform-random rows per column, values
  N(0,1) (the small parity LP m=500, n=1000, k=5; the adjoint LP
  m=50k, n=100k, k=8).
* ``planted_powerlaw``: column counts from a discrete power law
  P(k) ~ k^-alpha on [kmin, kmax], values N(0,1) * 10^U(-2,2) drawn per
  nonzero (m=200k, n=1M, nnz ~ 9.49M).
* ``multicommodity``: node-arc incidence blocks for K commodities on a
  random simple digraph plus per-node inflow capacity rows with slacks
  (150k nodes, 600k arcs, 8 commodities: m=1.35M, n=4.95M, nnz=14.55M).
* ``planted_coupled``: k rows per column among the first m-R rows plus R
  coupling rows with L distinct random columns each (m=5M, n=20M,
  k=5, R=50, L=200k: nnz=110M).
* ``tiny_dense``: small dense LPs with a planted optimum, for brute force.

Planted optimum (families with "planted"): x* has round(0.4 n) entries
U(0.1, 1) on a random support and 0 elsewhere; y* ~ N(0,1); z* ~ U(0.1, 1)
off the support of x* and 0 on it; b = A x*, c = A^T y* + z*.  Then
(x*, y*, z*) satisfies primal and dual feasibility and x*^T z* = 0, so
p* = c^T x* = b^T y*.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class LP:
    """Standard-form LP with CSR A, explicit CSR A^T, and optional plant."""
    m: int
    n: int
    a_rp: np.ndarray      # int64[m+1]
    a_ci: np.ndarray      # int32[nnz]
    a_v: np.ndarray       # float64[nnz]
    at_rp: np.ndarray     # int64[n+1]
    at_ci: np.ndarray     # int32[nnz]
    at_v: np.ndarray      # float64[nnz]
    b: np.ndarray         # float64[m]
    c: np.ndarray         # float64[n]
    x_star: Optional[np.ndarray] = None
    y_star: Optional[np.ndarray] = None
    z_star: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.a_v.shape[0])

    def dense(self) -> np.ndarray:
        """Dense copy of A (small problems only)."""
        A = np.zeros((self.m, self.n))
        rows = np.repeat(np.arange(self.m), np.diff(self.a_rp))
        A[rows, self.a_ci] = self.a_v
        return A

    def a_perm_to_at(self) -> np.ndarray:
        """perm[p] = position in A^T's arrays of A's p-th nonzero."""
        rows = np.repeat(np.arange(self.m, dtype=np.int64), np.diff(self.a_rp))
        key_a = self.a_ci.astype(np.int64) * self.m + rows
        order_t = np.argsort(key_a, kind="stable")
        perm = np.empty(self.nnz, dtype=np.int64)
        perm[order_t] = np.arange(self.nnz, dtype=np.int64)
        return perm


def _csr_pair(m: int, n: int, rows: np.ndarray, cols: np.ndarray,
              vals: np.ndarray, log=None):
    """CSR of A and of A^T from one coordinate list (entries distinct).
    log(msg), if given, is called after each stage (large inputs take
    minutes)."""
    rows = rows.astype(np.int64)
    cols = cols.astype(np.int64)
    key = rows * n + cols
    o = np.argsort(key, kind="stable")
    a_ci = cols[o].astype(np.int32)
    a_v = np.ascontiguousarray(vals[o], dtype=np.float64)
    a_rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=a_rp[1:])
    if log:
        log("CSR of A built")
    keyt = cols * m + rows
    ot = np.argsort(keyt, kind="stable")
    at_ci = rows[ot].astype(np.int32)
    at_v = np.ascontiguousarray(vals[ot], dtype=np.float64)
    at_rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=n), out=at_rp[1:])
    if log:
        log("CSR of A^T built")
    return a_rp, a_ci, a_v, at_rp, at_ci, at_v


def _distinct_rows_per_col(rng: np.random.Generator, counts: np.ndarray,
                           row_lo: int, row_hi: int):
    """For column j draw counts[j] distinct uniform rows in [row_lo, row_hi).

    Entries are drawn with replacement and duplicates inside a column are
    redrawn until none is left (vectorised rejection)."""
    n = counts.shape[0]
    nr = row_hi - row_lo
    if np.any(counts > nr):
        raise ValueError("column count exceeds the number of rows")
    cols = np.repeat(np.arange(n, dtype=np.int64), counts)
    rows = rng.integers(row_lo, row_hi, size=cols.shape[0], dtype=np.int64)
    while True:
        key = cols * nr + (rows - row_lo)
        o = np.argsort(key, kind="stable")
        ks = key[o]
        dup = np.zeros(ks.shape[0], dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            return cols, rows
        idx = o[dup]
        rows[idx] = rng.integers(row_lo, row_hi, size=idx.shape[0],
                                 dtype=np.int64)


def _plant(rng: np.random.Generator, lp_rows, lp_cols, lp_vals, m, n):
    """Planted optimum: returns (x*, y*, z*, b, c)."""
    x = np.zeros(n)
    k = int(round(0.4 * n))
    supp = rng.choice(n, size=k, replace=False)
    x[supp] = rng.uniform(0.1, 1.0, size=k)
    y = rng.standard_normal(m)
    z = np.zeros(n)
    off = np.ones(n, dtype=bool)
    off[supp] = False
    z[off] = rng.uniform(0.1, 1.0, size=int(off.sum()))
    # b = A x*, c = A^T y* + z*, accumulated in coordinate order
    b = np.bincount(lp_rows, weights=lp_vals * x[lp_cols], minlength=m)
    c = np.bincount(lp_cols, weights=lp_vals * y[lp_rows], minlength=n) + z
    return x, y, z, b, c


def planted_uniform(m: int = 500, n: int = 1000, k: int = 5,
                    seed: int = 0, name: str = "uniform") -> LP:
    """k distinct uniform rows per column, values N(0,1), planted optimum."""
    rng = np.random.default_rng(seed)
    counts = np.full(n, k, dtype=np.int64)
    cols, rows = _distinct_rows_per_col(rng, counts, 0, m)
    vals = rng.standard_normal(cols.shape[0])
    x, y, z, b, c = _plant(rng, rows, cols, vals, m, n)
    arrs = _csr_pair(m, n, rows, cols, vals)
    return LP(m, n, *arrs, b=b, c=c, x_star=x, y_star=y, z_star=z, name=name,
              meta=dict(family="uniform", k=k, seed=seed))


def powerlaw_counts(rng: np.random.Generator, n: int, alpha: float,
                    kmin: int, kmax: int) -> np.ndarray:
    """n draws of the discrete law P(k) proportional to k^-alpha on [kmin,kmax]."""
    ks = np.arange(kmin, kmax + 1, dtype=np.float64)
    p = ks ** (-alpha)
    p /= p.sum()
    return rng.choice(np.arange(kmin, kmax + 1), size=n, p=p).astype(np.int64)


def planted_powerlaw(m: int = 200_000, n: int = 1_000_000, alpha: float = 2.1,
                     kmin: int = 2, kmax: int = 5000, seed: int = 1,
                     name: str = "powerlaw") -> LP:
    """Power-law column counts, values N(0,1)*10^U(-2,2), planted optimum."""
    rng = np.random.default_rng(seed)
    counts = powerlaw_counts(rng, n, alpha, kmin, min(kmax, m))
    cols, rows = _distinct_rows_per_col(rng, counts, 0, m)
    nnz = cols.shape[0]
    vals = rng.standard_normal(nnz) * 10.0 ** rng.uniform(-2.0, 2.0, size=nnz)
    x, y, z, b, c = _plant(rng, rows, cols, vals, m, n)
    arrs = _csr_pair(m, n, rows, cols, vals)
    return LP(m, n, *arrs, b=b, c=c, x_star=x, y_star=y, z_star=z, name=name,
              meta=dict(family="powerlaw", alpha=alpha, kmin=kmin, kmax=kmax,
                        seed=seed))


def _random_simple_digraph(rng: np.random.Generator, nodes: int, arcs: int):
    """Distinct (tail, head) pairs, tail != head, uniform."""
    if arcs > nodes * (nodes - 1):
        raise ValueError("too many arcs")
    tail = rng.integers(0, nodes, size=arcs, dtype=np.int64)
    head = rng.integers(0, nodes - 1, size=arcs, dtype=np.int64)
    head = head + (head >= tail)            # uniform over heads != tail
    while True:
        key = tail * nodes + head
        o = np.argsort(key, kind="stable")
        ks = key[o]
        dup = np.zeros(arcs, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        idx = o[dup]
        tail[idx] = rng.integers(0, nodes, size=idx.shape[0], dtype=np.int64)
        h = rng.integers(0, nodes - 1, size=idx.shape[0], dtype=np.int64)
        head[idx] = h + (h >= tail[idx])
    return tail, head


def multicommodity(nodes: int = 150_000, arcs: int = 600_000,
                   commodities: int = 8, seed: int = 2,
                   name: str = "mcf") -> LP:
    """Multicommodity-flow LP with per-node inflow capacity rows and slacks.

    Variables: f[k, a] (commodity-major, k*arcs + a) then slack s[v].
    Rows: conservation (k, v) at k*nodes + v: sum_out f - sum_in f = supply;
    then capacity row v: sum_k sum_{a into v} f[k,a] + s[v] = u[v].
    Supplies come from a planted flow f* ~ U(0,1) on a random 20% of the
    arcs of each commodity; u ~ U(10,1000) raised to 1.1 * planted inflow,
    so the LP is feasible; costs U(1,100) (slack cost 0) keep it bounded.
    The optimum is not planted."""
    rng = np.random.default_rng(seed)
    tail, head = _random_simple_digraph(rng, nodes, arcs)
    K = commodities
    m = K * nodes + nodes
    n = K * arcs + nodes
    kk = np.repeat(np.arange(K, dtype=np.int64), arcs)
    aa = np.tile(np.arange(arcs, dtype=np.int64), K)
    var = kk * arcs + aa
    r_tail = kk * nodes + tail[aa]
    r_head = kk * nodes + head[aa]
    r_cap = K * nodes + head[aa]
    s_var = K * arcs + np.arange(nodes, dtype=np.int64)
    s_row = K * nodes + np.arange(nodes, dtype=np.int64)
    rows = np.concatenate([r_tail, r_head, r_cap, s_row])
    cols = np.concatenate([var, var, var, s_var])
    vals = np.concatenate([np.ones(K * arcs), -np.ones(K * arcs),
                           np.ones(K * arcs), np.ones(nodes)])
    fstar = np.zeros(K * arcs)
    for k in range(K):
        sel = rng.choice(arcs, size=int(round(0.2 * arcs)), replace=False)
        fstar[k * arcs + sel] = rng.uniform(0.0, 1.0, size=sel.shape[0])
    supply = (np.bincount(r_tail, weights=fstar, minlength=K * nodes)
              - np.bincount(r_head, weights=fstar, minlength=K * nodes))
    inflow = np.bincount(head[aa], weights=fstar, minlength=nodes)
    u = np.maximum(rng.uniform(10.0, 1000.0, size=nodes), 1.1 * inflow)
    b = np.concatenate([supply, u])
    c = np.concatenate([rng.uniform(1.0, 100.0, size=K * arcs),
                        np.zeros(nodes)])
    arrs = _csr_pair(m, n, rows, cols, vals)
    return LP(m, n, *arrs, b=b, c=c, name=name,
              meta=dict(family="mcf", nodes=nodes, arcs=arcs, K=K, seed=seed))


def planted_coupled(m: int = 5_000_000, n: int = 20_000_000, k: int = 5,
                    n_coupling: int = 50, coupling_len: int = 200_000,
                    seed: int = 4, name: str = "coupled", log=None) -> LP:
    """k distinct rows per column among the first m-R rows, plus R coupling
    rows (the last R rows) each with L distinct random columns; values
    N(0,1); planted optimum.  log(msg), if given, reports each stage."""
    rng = np.random.default_rng(seed)
    counts = np.full(n, k, dtype=np.int64)
    cols, rows = _distinct_rows_per_col(rng, counts, 0, m - n_coupling)
    if log:
        log("column entries drawn")
    crow, ccol = [], []
    for r in range(n_coupling):
        cc = rng.choice(n, size=coupling_len, replace=False)
        ccol.append(cc.astype(np.int64))
        crow.append(np.full(coupling_len, m - n_coupling + r, dtype=np.int64))
    if n_coupling:
        rows = np.concatenate([rows] + crow)
        cols = np.concatenate([cols] + ccol)
    vals = rng.standard_normal(cols.shape[0])
    x, y, z, b, c = _plant(rng, rows, cols, vals, m, n)
    if log:
        log("coupling rows drawn, optimum planted")
    arrs = _csr_pair(m, n, rows, cols, vals, log)
    return LP(m, n, *arrs, b=b, c=c, x_star=x, y_star=y, z_star=z, name=name,
              meta=dict(family="coupled", k=k, R=n_coupling, L=coupling_len,
                        seed=seed))


def planted_flat(m: int = 300, n: int = 1000, k: int = 5, seed: int = 1) -> LP:
    """The uniform pattern with c = A^T y* (no reduced costs): c^T x = y*^T b
    on the whole feasible set, so every feasible point is optimal.  b = A x*
    with x* ~ U(0.1, 1) strictly positive."""
    base = planted_uniform(m=m, n=n, k=k, seed=seed)
    rows = np.repeat(np.arange(m), np.diff(base.a_rp))
    cols = base.a_ci.astype(np.int64)
    rng = np.random.default_rng(seed + 100)
    x = rng.uniform(0.1, 1.0, n)
    y = rng.standard_normal(m)
    b = np.bincount(rows, weights=base.a_v * x[cols], minlength=m)
    c = np.bincount(cols, weights=base.a_v * y[rows], minlength=n)
    arrs = _csr_pair(m, n, rows, cols, base.a_v)
    return LP(m, n, *arrs, b=b, c=c, x_star=x, y_star=y, z_star=np.zeros(n),
              name="flat", meta=dict(family="flat", k=k, seed=seed))


def tiny_dense(m: int, n: int, seed: int, density: float = 1.0) -> LP:
    """Small LP (dense or sparse pattern) with a planted optimum."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    for j in range(n):                      # every column gets an entry
        if not mask[:, j].any():
            mask[rng.integers(0, m), j] = True
    rows, cols = np.nonzero(mask)
    vals = rng.standard_normal(rows.shape[0])
    x, y, z, b, c = _plant(rng, rows, cols, vals, m, n)
    arrs = _csr_pair(m, n, rows, cols, vals)
    return LP(m, n, *arrs, b=b, c=c, x_star=x, y_star=y, z_star=z,
              name=f"tiny{m}x{n}", meta=dict(family="tiny", seed=seed))


def from_coo(m: int, n: int, rows, cols, vals, b, c, name="coo") -> LP:
    """LP from a user coordinate list (entries must be distinct)."""
    arrs = _csr_pair(m, n, np.asarray(rows), np.asarray(cols),
                     np.asarray(vals, dtype=np.float64))
    return LP(m, n, *arrs, b=np.asarray(b, dtype=np.float64),
              c=np.asarray(c, dtype=np.float64), name=name)


# The five workloads at full size, and a scale knob for parity-sized copies.
WORKLOADS = {
    "uniform_m500_n1k": dict(fn=planted_uniform, kw=dict(m=500, n=1000, k=5, seed=0)),
    "powerlaw_m200k_n1m": dict(fn=planted_powerlaw, kw=dict(m=200_000, n=1_000_000, seed=1)),
    "mcf_150knodes_600karcs_k8": dict(fn=multicommodity, kw=dict(nodes=150_000, arcs=600_000, commodities=8, seed=2)),
    "uniform_m50k_n100k_k8": dict(fn=planted_uniform, kw=dict(m=50_000, n=100_000, k=8, seed=3)),
    "coupled_m5m_n20m": dict(fn=planted_coupled, kw=dict(m=5_000_000, n=20_000_000, seed=4)),
}


def make(workload: str, **override) -> LP:
    w = WORKLOADS[workload]
    kw = dict(w["kw"])
    kw.update(override)
    lp = w["fn"](**kw)
    lp.name = workload
    return lp


def target_vector(n: int, seed: int) -> np.ndarray:
    """x_target ~ U(0,1) for the unrolled-loss workload."""
    return np.random.default_rng(seed + 1000).uniform(0.0, 1.0, size=n)
