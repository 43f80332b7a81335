"""GPU parity of the HIP path against the FP64 CPU oracle (through the C ABI).

Bars: bitwise for the Ruiz factors and for integer-valued SpMVs; 1e-10
relative per iteration on the iterates over the first 100 iterations; 1e-12
absolute on the final relative KKT errors; same iteration counts, restarts
and snapshot points.
"""
import threading
import time

import numpy as np
import pytest

from paper_2510_24429_amd import lpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    import torch
    assert torch.cuda.is_available()
    from paper_2510_24429_amd.solver import Solver as S
    return S


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def elem(a, b):
    """Largest entry-wise difference relative to the largest entry of b: a
    single wrong entry shows here even when the norm-wise error is small."""
    s = np.max(np.abs(b)) if b.size else 0.0
    return np.max(np.abs(a - b)) / (s if s > 0 else 1.0) if a.size else 0.0


def err(a, b):
    return max(rel(a, b), elem(a, b))


def _integer_lp(seed=0):
    """Integer-valued CSR spanning every bin: empty rows, short rows, rows
    between the tiles, single-workgroup rows and rows long enough to split."""
    rng = np.random.default_rng(seed)
    m, n = 3000, 40000
    lens = np.concatenate([
        np.zeros(50, dtype=np.int64),
        rng.integers(1, 17, 2000),
        rng.integers(17, 1025, 800),
        np.array([1023, 1024, 1025, 2047, 2048, 2049, 4096, 4097]),
        rng.integers(4098, 9000, 40),
        np.array([20000, 30001, 39999]),
    ])
    lens = lens[:m] if lens.shape[0] >= m else np.concatenate(
        [lens, rng.integers(0, 8, m - lens.shape[0])])
    rng.shuffle(lens)
    rows, cols = [], []
    for i, L in enumerate(lens):
        c = rng.choice(n, size=int(L), replace=False)
        rows.append(np.full(int(L), i))
        cols.append(c)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = rng.integers(-3, 4, rows.shape[0]).astype(np.float64)
    vals[vals == 0] = 1.0
    return lpgen.from_coo(m, n, rows, cols, vals, np.ones(m), np.ones(n), name="int")


PANELS = {"panels_a": 4, "panels_at": 8}


@pytest.mark.parametrize("panels", [False, True])
@pytest.mark.parametrize("split", [False, True])
def test_spmv_bins_bitwise_on_integers(Solver, split, panels):
    lp = _integer_lp()
    tuning = {"split_threshold": 4096, "split_chunk": 1000} if split else {}
    if panels:
        tuning.update(PANELS)
    # both streamed-load kinds: non-temporal with panels, plain without
    tuning["stream_nt"] = 1 if panels else 0
    s = Solver.from_lp(lp, tuning=tuning)
    assert (s.panel_count(0), s.panel_count(1)) == ((4, 8) if panels else (1, 1))
    st = s.bin_stats(0)
    assert st[0] > 0 and st[1] > 0
    if split:
        assert st[2] > 0
    rng = np.random.default_rng(1)
    x = rng.integers(-5, 6, lp.n).astype(np.float64)
    y = rng.integers(-5, 6, lp.m).astype(np.float64)
    A = lp.dense()
    ax = A @ x      # integers well below 2^24: exact in any order
    aty = A.T @ y
    assert np.array_equal(s.spmv(0, x), ax)
    assert np.array_equal(s.spmv(1, y), aty)
    assert np.array_equal(s.spmv(0, x, precision=1), ax)
    assert np.array_equal(s.spmv(1, y, precision=1), aty)
    # before configure the scaled matrix is A itself (unit factors); the
    # scaled values take the panel path when the side is panelled
    assert np.array_equal(s.spmv(0, x, scaled=True), ax)
    assert np.array_equal(s.spmv(1, y, scaled=True), aty)
    assert np.array_equal(s.spmv(0, x, scaled=True, precision=1), ax)
    assert np.array_equal(s.spmv(1, y, scaled=True, precision=1), aty)
    # after configure the scaled values differ from the loaded ones; the
    # loaded-value products (also the FP32 ones, whose panel copy is swapped
    # in for the call) stay A x and A^T y, and the scaled ones are restored
    s.configure(eps_rel=1e-6)
    sc0 = s.spmv(0, x, scaled=True, precision=1)
    for prec in (0, 1):
        assert np.array_equal(s.spmv(0, x, precision=prec), ax)
        assert np.array_equal(s.spmv(1, y, precision=prec), aty)
    assert np.array_equal(s.spmv(0, x, scaled=True, precision=1), sc0)
    s.close()


def test_ruiz_factors_bitwise(Solver, oracle):
    for lp in (lpgen.make("uniform_m500_n1k"),
               lpgen.planted_powerlaw(m=2000, n=10000, kmax=1500, seed=7)):
        dr, dc, _ = oracle.ruiz(lp, 10)
        with Solver.from_lp(lp) as s:
            s.configure(ruiz_passes=10, power_iters=5)
            gdr, gdc = s.get_scaling()
        assert np.array_equal(gdr, dr)
        assert np.array_equal(gdc, dc)


def test_power_iteration_matches(Solver, oracle):
    lp = lpgen.make("uniform_m500_n1k")
    ref = oracle.solve(lp, eps_rel=1e-6, max_iters=0)
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-6)
        inf = s.info()
    assert abs(inf["sigma_hat"] - ref.info["sigma_hat"]) <= 1e-13 * ref.info["sigma_hat"]
    assert abs(inf["omega0"] - ref.info["omega0"]) <= 1e-13 * ref.info["omega0"]


def _trace_parity(Solver, oracle, lp, K, l=None, tuning=None, **kw):
    ref = oracle.solve(lp, l=l, trace_k=K, **kw)
    worst = 0.0
    with Solver.from_lp(lp, lb=l, tuning=tuning) as s:
        s.configure(**kw)
        for k in range(K):
            s.iterate(1)
            x, y, _ = s.get_iterate()
            worst = max(worst, err(x, ref.trace_x[k]), err(y, ref.trace_y[k]))
    return worst


@pytest.mark.parametrize("variant", [0, 1])
def test_iterates_first_100_match_oracle(Solver, oracle, variant):
    lp = lpgen.make("uniform_m500_n1k")
    worst = _trace_parity(Solver, oracle, lp, 100, eps_rel=1e-8, variant=variant)
    assert worst <= 1e-10, worst


def test_iterates_match_with_eval_every_iteration(Solver, oracle):
    # Algorithm 1 tests maxresid before every iteration: eval_every = 1
    lp = lpgen.make("uniform_m500_n1k")
    worst = _trace_parity(Solver, oracle, lp, 60, eps_rel=1e-8, eval_every=1)
    assert worst <= 1e-10, worst


@pytest.mark.parametrize("panels", [False, True])
@pytest.mark.parametrize("variant", [0, 1])
def test_iterates_match_with_lower_bounds(Solver, oracle, variant, panels):
    lp = lpgen.planted_uniform(m=800, n=2500, k=6, seed=12)
    l = -np.random.default_rng(12).uniform(0.0, 0.5, lp.n)
    worst = _trace_parity(Solver, oracle, lp, 100, l=l, eps_rel=1e-8, eval_every=16,
                          variant=variant, tuning=PANELS if panels else None)
    assert worst <= 1e-10, worst


@pytest.mark.parametrize("panels", [False, True])
@pytest.mark.parametrize("variant", [0, 1])
def test_iterates_match_multi_tile_ragged(Solver, oracle, variant, panels):
    # several tiles per kernel, a ragged last block, short and long rows
    lp = lpgen.planted_powerlaw(m=3000, n=20000, kmax=2500, seed=21)
    worst = _trace_parity(Solver, oracle, lp, 100, eps_rel=1e-8, eval_every=32,
                          variant=variant, tuning=PANELS if panels else None)
    assert worst <= 1e-10, worst


LAYOUTS = [{"block_rows": 0}, {"block_rows": 64},
           {"sort_rows": 0, "sort_cols": 0},
           {"sort_rows": 1, "sort_cols": 1, "panels_a": 4, "panels_at": 2}]


@pytest.mark.parametrize("tuning", LAYOUTS, ids=["rows_tile", "rows_64", "unsorted", "sorted_panels"])
def test_iterates_match_with_layout_keys(Solver, oracle, tuning):
    # the internal order and the row-block shapes change only rounding
    lp = lpgen.planted_powerlaw(m=3000, n=20000, kmax=2500, seed=21)
    worst = _trace_parity(Solver, oracle, lp, 100, eps_rel=1e-8, eval_every=32,
                          variant=1, tuning=tuning)
    assert worst <= 1e-10, worst


@pytest.mark.parametrize("variant", [0, 1])
def test_iterates_match_block_structured_panels(Solver, oracle, variant):
    # commodity-major columns cut into 8 panels: a conservation row's entries
    # lie in one or two panels, so most stacked rows are empty and skipped
    lp = lpgen.multicommodity(nodes=1500, arcs=6000, commodities=8, seed=5)
    with Solver.from_lp(lp, tuning={"panels_a": 8, "panels_at": 4}) as s:
        assert s.panel_count(0) == 8 and s.panel_count(1) == 4
    # the iteration limit lies past the traced window; it only ends the
    # oracle's run early
    worst = _trace_parity(Solver, oracle, lp, 100, eps_rel=1e-8, eval_every=32,
                          max_iters=101, variant=variant,
                          tuning={"panels_a": 8, "panels_at": 4})
    assert worst <= 1e-10, worst


@pytest.mark.parametrize("precision", [0, 1])
def test_panelled_fp32_and_fp64_steps_match_plain(Solver, precision):
    # the panel path changes only the summation order of each row: iterates
    # stay within rounding of the unpanelled path in both precisions
    lp = lpgen.planted_powerlaw(m=3000, n=20000, kmax=2500, seed=22)
    out = []
    for tuning in (None, PANELS):
        with Solver.from_lp(lp, tuning=tuning) as s:
            s.configure(eps_rel=1e-12, precision=precision, eval_every=1024)
            s.iterate(200)
            out.append(s.get_iterate()[:2])
    tol = 1e-11 if precision == 0 else 1e-4
    assert rel(out[1][0], out[0][0]) <= tol and rel(out[1][1], out[0][1]) <= tol


def _solve_both(Solver, oracle, lp, levels, eps, tuning=None, **kw):
    ref = oracle.solve(lp, levels=levels, eps_rel=eps, keep_snap_vectors=True, **kw)
    s = Solver.from_lp(lp, tuning=tuning)
    s.configure(levels=levels, eps_rel=eps, **kw)
    st = s.solve()
    return ref, s, st


@pytest.mark.parametrize("variant,panels", [(0, False), (1, False), (1, True)])
def test_full_solve_kkt_and_snapshots(Solver, oracle, variant, panels):
    lp = lpgen.make("uniform_m500_n1k")
    levels = [1e-4, 1e-6]
    ref, s, st = _solve_both(Solver, oracle, lp, levels, 1e-6, variant=variant,
                             tuning=PANELS if panels else None)
    inf = s.info()
    assert st == 1 and ref.info["status"] == 1
    assert inf["iters"] == ref.info["iters"]
    assert inf["restarts"] == ref.info["restarts"]
    for key in ("rel_p", "rel_d", "rel_gap", "maxresid"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
    assert abs(inf["kkt"]["pobj"] - ref.kkt["pobj"]) <= 1e-9 * (1 + abs(ref.kkt["pobj"]))
    log = s.eval_log()
    assert np.array_equal(log[:, 0], ref.eval_log[:, 0])
    assert np.array_equal(log[:, 5], ref.eval_log[:, 5])          # restarts
    assert s.snapshot_count() == len(ref.snaps) == 2
    for i, sn in enumerate(ref.snaps):
        info, x, y, z = s.snapshot(i)
        assert s.snapshot_info(i) == info           # the call without vectors
        assert info["level"] == sn["level"] and info["iter"] == sn["iter"]
        assert abs(info["maxresid"] - sn["maxresid"]) <= 1e-12
        assert err(x, ref.snap_x[i]) <= 1e-8 and err(y, ref.snap_y[i]) <= 1e-8
        assert np.max(np.abs(z - ref.snap_z[i])) <= 1e-8 * (1 + np.max(np.abs(ref.snap_z[i])))
        # the snapshot satisfies the level on the original data (CPU recompute)
        kk = oracle.kkt(lp, x, y)
        assert kk["maxresid"] <= sn["level"]
    s.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_pid_primal_weight_matches_oracle(Solver, oracle, variant):
    lp = lpgen.make("uniform_m500_n1k")
    kw = dict(variant=variant, omega_rule=1, eval_every=32)
    ref, s, st = _solve_both(Solver, oracle, lp, [1e-4], 1e-8, **kw)
    inf = s.info()
    assert st == 1 and ref.info["status"] == 1
    assert inf["iters"] == ref.info["iters"]
    assert inf["restarts"] == ref.info["restarts"]
    # the PID sets log omega from log(dx / dy) of the late restart intervals,
    # where the paths' rounding-level differences in the iterates are
    # relatively largest; the decisions (restart points) must agree exactly
    assert abs(np.log(inf["omega"]) - np.log(ref.info["omega"])) <= 1e-6
    for key in ("rel_p", "rel_d", "rel_gap", "maxresid"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
    log = s.eval_log()
    assert np.array_equal(log[:, 5], ref.eval_log[:, 5])          # restarts
    s.close()


def test_full_solve_alg1_schedule_1e8(Solver, oracle):
    lp = lpgen.make("uniform_m500_n1k")
    levels = oracle.alg1_levels(1e-2, 1e-8)
    ref, s, st = _solve_both(Solver, oracle, lp, levels, 1e-8, literal_snapshots=1)
    assert st == 1
    got = [s.snapshot(i)[0] for i in range(s.snapshot_count())]
    assert [g["level"] for g in got] == [r["level"] for r in ref.snaps] == levels
    assert [g["iter"] for g in got] == [r["iter"] for r in ref.snaps]
    inf = s.info()
    for key in ("rel_p", "rel_d", "rel_gap"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12
    s.close()


def test_graph_and_stream_paths_agree(Solver):
    lp = lpgen.planted_uniform(m=4000, n=9000, k=5, seed=31)
    out = []
    for g in (0, 1):
        with Solver.from_lp(lp) as s:
            s.configure(eps_rel=1e-7, use_graph=g)
            st = s.solve()
            x, y, _ = s.get_iterate()
            out.append((st, s.info()["iters"], x, y))
    assert out[0][0] == out[1][0] and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2]) and np.array_equal(out[0][3], out[1][3])


def test_status_iter_limit_numerical_warm_start(Solver):
    lp = lpgen.make("uniform_m500_n1k")
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-12, max_iters=100)
        assert s.solve() == 2
        assert s.info()["iters"] == 100
    b = lp.b.copy()
    b[3] = np.nan
    lpn = lpgen.LP(lp.m, lp.n, lp.a_rp, lp.a_ci, lp.a_v, lp.at_rp, lp.at_ci, lp.at_v, b, lp.c)
    with Solver.from_lp(lpn) as s:
        s.configure(eps_rel=1e-6, max_iters=1000)
        assert s.solve() == 5
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-6, levels=[1e-4, 1e-6])
        s.set_iterate(lp.x_star, lp.y_star)
        assert s.solve() == 1
        assert s.info()["iters"] == 0 and s.snapshot_count() == 2


def test_cancel_and_time_limit(Solver):
    lp = lpgen.planted_uniform(m=20000, n=60000, k=5, seed=4)
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-14, time_limit_s=0.5)
        assert s.solve() == 3
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-14)
        threading.Timer(0.3, s.cancel).start()
        t0 = time.time()
        assert s.solve() == 4
        assert time.time() - t0 < 30


def test_snapshot_callback(Solver, oracle):
    """The callback receives each snapshot's info and its unscaled vectors,
    equal to what pdhg_snapshot returns, in emission order, also on a second
    solve of the same context (the host copies are reused)."""
    lp = lpgen.make("uniform_m500_n1k")
    levels = [1e-2, 1e-4, 1e-6]
    with Solver.from_lp(lp) as s:
        for rnd in range(2):
            seen = []
            ev = threading.Event()

            def cb(idx, info, x, y, z):
                seen.append((idx, info, x, y, z))
                if len(seen) == 3:
                    ev.set()

            s.configure(eps_rel=1e-6, levels=levels)
            s.set_snapshot_callback(cb, with_vectors=True)
            assert s.solve() == 1
            assert ev.wait(10)
            assert [(i, inf["level"]) for i, inf, *_ in seen] == list(enumerate(levels))
            for idx, info, x, y, z in seen:
                ref_info, rx, ry, rz = s.snapshot(idx)
                assert info == ref_info
                assert np.array_equal(x, rx) and np.array_equal(y, ry)
                assert np.array_equal(z, rz)
                assert oracle.kkt(lp, x, y)["maxresid"] <= info["level"]


def test_bad_inputs_rejected(Solver):
    from paper_2510_24429_amd._lib import PDHGError
    lp = lpgen.make("uniform_m500_n1k")
    at_v = lp.at_v.copy()
    at_v[0] += 1.0
    with pytest.raises(PDHGError, match="TRANSPOSE"):
        Solver(lp.m, lp.n, lp.a_rp, lp.a_ci, lp.a_v, lp.at_rp, lp.at_ci, at_v, lp.b, lp.c)
    with Solver.from_lp(lp) as s:
        with pytest.raises(PDHGError, match="STATE"):
            s.iterate(1)
        with pytest.raises(PDHGError, match="ARG"):
            s.configure(levels=[1e-6, 1e-4])


def _full_size_windows(Solver, oracle, lp, panels, kw, K_step, K_graph,
                       tag, graph_every=64):
    """Full-size parity in the benchmark's launch configuration (column
    panels and streamed-load kind chosen from the sizes):
      - Ruiz factors bitwise;
      - K_step single iterations (no graph), each iterate element-wise
        within 1e-10 of the oracle's, with their evaluations and restart
        decisions at eval_every = 2;
      - K_graph iterations as replayed batches of graph_every iterations
        (the graph the benchmark times, with its in-graph evaluation and
        restart; the benchmark's batch is 64), the iterate after the last
        batch element-wise within 1e-10 and the evaluation log's restart
        flags equal."""
    dr, dc, _ = oracle.ruiz(lp, 10)
    print(f"[full-size] {tag}: oracle runs", flush=True)
    kw1 = dict(kw, eval_every=2)
    ref1 = oracle.solve(lp, trace_k=K_step, max_iters=K_step, **kw1)
    kw2 = dict(kw, eval_every=graph_every)
    print(f"[full-size] {tag}: oracle run of {K_graph} iterations", flush=True)
    ref2 = oracle.solve(lp, max_iters=K_graph, **kw2)
    with Solver.from_lp(lp) as s:
        assert (s.panel_count(0), s.panel_count(1)) == panels
        s.configure(**kw1)
        gdr, gdc = s.get_scaling()
        assert np.array_equal(gdr, dr) and np.array_equal(gdc, dc)
        print(f"[full-size] {tag}: {K_step} single steps", flush=True)
        for k in range(K_step):
            s.iterate(1)
            x, y, _ = s.get_iterate()
            assert err(x, ref1.trace_x[k]) <= 1e-10, k
            assert err(y, ref1.trace_y[k]) <= 1e-10, k
        log = s.eval_log()
        assert np.array_equal(log[:, 5], ref1.eval_log[:, 5])
        assert np.allclose(log[:, 1:5], ref1.eval_log[:, 1:5], rtol=1e-9, atol=0,
                           equal_nan=True)
        print(f"[full-size] {tag}: {K_graph} iterations in graph batches", flush=True)
        s.configure(**kw2)
        s.iterate(K_graph)
        x, y, _ = s.get_iterate()
        log = s.eval_log()
    assert log.shape[0] == ref2.eval_log.shape[0] == K_graph // graph_every + 1
    assert np.array_equal(log[:, 0], ref2.eval_log[:, 0])
    assert np.array_equal(log[:, 5], ref2.eval_log[:, 5])
    assert np.allclose(log[:, 1:5], ref2.eval_log[:, 1:5], rtol=1e-9, atol=0,
                       equal_nan=True)
    assert err(x, ref2.x) <= 1e-10, err(x, ref2.x)
    assert err(y, ref2.y) <= 1e-10, err(y, ref2.y)


@pytest.mark.timeout(900)
def test_full_size_multicommodity_parity(Solver, oracle):
    """The multicommodity workload at full size (m=1.35M, n=4.95M,
    nnz=14.55M): 8 column panels for the dual step, non-temporal streaming.
    The step size and primal weight are computed (power iteration)."""
    lp = lpgen.make("mcf_150knodes_600karcs_k8")
    _full_size_windows(Solver, oracle, lp, (8, 1),
                       dict(eps_rel=1e-8, variant=1), 4, 64, "multicommodity")


@pytest.mark.timeout(900)
def test_full_size_coupled_parity(Solver, oracle):
    """The largest workload at full size (m=5M, n=20M, nnz=110M): 8 column
    panels for the dual step, 4 for the primal step, non-temporal streaming.
    The serial oracle takes seconds per iteration here, so the step size and
    primal weight are fixed (no 100-step power iteration) and the graph
    window is two batches of 8 iterations."""
    lp = lpgen.make("coupled_m5m_n20m")
    _full_size_windows(Solver, oracle, lp, (8, 4),
                       dict(eps_rel=1e-8, variant=1, eta=0.5, omega0=1.3), 3, 16,
                       "coupled", graph_every=8)


@pytest.mark.timeout(900)
def test_full_size_powerlaw_parity(Solver, oracle):
    """The power-law workload at full size (m=200k, n=1M, nnz~9.4M):
    power-iteration estimate and initial primal weight within 1e-13 of the
    oracle's; the first 100 iterations (both variants' bench default, the
    Halpern one, with one evaluation at 64) element-wise within 1e-10;
    128 iterations as two replayed graph batches."""
    lp = lpgen.make("powerlaw_m200k_n1m")
    kw = dict(eps_rel=1e-8, variant=1)
    dr, dc, _ = oracle.ruiz(lp, 10)
    K = 100
    print("[full-size] power-law: oracle run", flush=True)
    ref = oracle.solve(lp, trace_k=K, max_iters=128, **kw)
    with Solver.from_lp(lp) as s:
        assert (s.panel_count(0), s.panel_count(1)) == (4, 1)
        s.configure(**kw)
        inf = s.info()
        for key in ("sigma_hat", "omega0", "eta"):
            assert abs(inf[key] - ref.info[key]) <= 1e-13 * abs(ref.info[key]), key
        gdr, gdc = s.get_scaling()
        assert np.array_equal(gdr, dr) and np.array_equal(gdc, dc)
        print("[full-size] power-law: 100 single steps", flush=True)
        for k in range(K):
            s.iterate(1)
            x, y, _ = s.get_iterate()
            assert err(x, ref.trace_x[k]) <= 1e-10, k
            assert err(y, ref.trace_y[k]) <= 1e-10, k
        s.iterate(128 - K)
        x, y, _ = s.get_iterate()
        assert err(x, ref.x) <= 1e-10 and err(y, ref.y) <= 1e-10
        log1 = s.eval_log()
        print("[full-size] power-law: 128 iterations in graph batches", flush=True)
        s.configure(**kw)
        s.iterate(128)
        x, y, _ = s.get_iterate()
        log2 = s.eval_log()
    for log in (log1, log2):
        assert log.shape == ref.eval_log.shape
        assert np.array_equal(log[:, 0], ref.eval_log[:, 0])
        assert np.array_equal(log[:, 5], ref.eval_log[:, 5])
        assert np.allclose(log[:, 1:5], ref.eval_log[:, 1:5], rtol=1e-9, atol=0)
    assert err(x, ref.x) <= 1e-10 and err(y, ref.y) <= 1e-10


@pytest.mark.timeout(900)
def test_mid_size_full_solve_parity(Solver, oracle):
    """A full solve of a 20k x 60k LP (8 nonzeros per column, about 5.5k and
    11k iterations) in both variants: the same iteration count, restarts and
    snapshot iterations as the oracle, final relative KKT errors within
    1e-12."""
    lp = lpgen.planted_uniform(m=20_000, n=60_000, k=8, seed=31)
    for variant in (0, 1):
        levels = [1e-3, 1e-5]
        ref = oracle.solve(lp, levels=levels, eps_rel=1e-6, variant=variant)
        with Solver.from_lp(lp) as s:
            s.configure(levels=levels, eps_rel=1e-6, variant=variant)
            st = s.solve()
            inf = s.info()
            log = s.eval_log()
            snaps = [s.snapshot(i)[0] for i in range(s.snapshot_count())]
        print(f"[mid-size] variant {variant}: {inf['iters']} iterations, "
              f"{inf['restarts']} restarts (oracle {ref.info['iters']}, "
              f"{ref.info['restarts']})", flush=True)
        assert st == 1 and ref.info["status"] == 1
        assert inf["iters"] == ref.info["iters"]
        assert inf["restarts"] == ref.info["restarts"]
        assert np.array_equal(log[:, 5], ref.eval_log[:, 5])
        for key in ("rel_p", "rel_d", "rel_gap", "maxresid"):
            assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
        assert [(sn["level"], sn["iter"]) for sn in snaps] == \
            [(sn["level"], sn["iter"]) for sn in ref.snaps]


# ------------------------------------------------- feasibility polishing

def _solve_pair(Solver, oracle, lp, **kw):
    ref = oracle.solve(lp, **kw)
    s = Solver.from_lp(lp)
    s.configure(**kw)
    st = s.solve()
    return ref, s, st


@pytest.mark.parametrize("mode", [1, 2])
def test_feasibility_stop_measures_match_oracle(Solver, oracle, mode):
    lp = lpgen.make("uniform_m500_n1k")
    ref, s, st = _solve_pair(Solver, oracle, lp, eps_rel=1e-6, stop_on=mode)
    inf = s.info()
    assert st == 1 and ref.info["status"] == 1
    assert inf["iters"] == ref.info["iters"] and inf["restarts"] == ref.info["restarts"]
    key = "rel_p" if mode == 1 else "rel_d"
    assert inf["kkt"][key] <= 1e-6
    assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12
    s.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_failed_polishing_leaves_the_solve_unchanged(Solver, oracle, variant):
    # attempts that fail must not alter the main iteration; their count and
    # phase iterations match the oracle's
    lp = lpgen.planted_powerlaw(m=1500, n=6000, kmax=600, seed=3)
    ref, s, st = _solve_pair(Solver, oracle, lp, eps_rel=1e-6, variant=variant, polish=1)
    inf = s.info()
    assert st == 1 and ref.info["status"] == 1
    assert inf["polish_attempts"] == ref.info["polish_attempts"] >= 1
    assert inf["polish_iters"] == ref.info["polish_iters"]
    assert inf["candidate"] != 2
    assert inf["iters"] == ref.info["iters"] and inf["restarts"] == ref.info["restarts"]
    for key in ("rel_p", "rel_d", "rel_gap", "maxresid"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
    with Solver.from_lp(lp) as s0:
        s0.configure(eps_rel=1e-6, variant=variant)
        assert s0.solve() == 1
        assert s0.info()["iters"] == inf["iters"]
    s.close()


def test_polishing_success_matches_oracle(Solver, oracle):
    lp = lpgen.planted_flat(300, 1000, 5, 1)
    ref, s, st = _solve_pair(Solver, oracle, lp, eps_rel=1e-8, variant=0, polish=1)
    inf = s.info()
    assert st == 1 and ref.info["candidate"] == 2 and inf["candidate"] == 2
    assert inf["iters"] == ref.info["iters"]
    assert inf["polish_attempts"] == ref.info["polish_attempts"]
    assert inf["polish_iters"] == ref.info["polish_iters"]
    for key in ("rel_p", "rel_d", "rel_gap", "maxresid"):
        assert abs(inf["kkt"][key] - ref.kkt[key]) <= 1e-12, key
    x, y, _ = s.get_iterate()
    assert err(x, ref.x) <= 1e-10 and err(y, ref.y) <= 1e-10
    kk = oracle.kkt(lp, x, y)
    assert kk["maxresid"] <= 1e-8
    s.close()


def test_residuals_of_the_better_candidate(Solver, oracle):
    lp = lpgen.make("uniform_m500_n1k")
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-12, eval_every=64)
        s.iterate(100)                     # mid-way between evaluations
        k0, k1, kb = s.residuals(0), s.residuals(1), s.residuals(2)
    want = k1 if k1["maxresid"] < k0["maxresid"] else k0
    assert kb["maxresid"] == want["maxresid"] and kb["candidate"] == want["candidate"]
