"""GPU checks of the FP32 bulk + FP64 refinement path and of the unrolled
adjoint, against the FP64 CPU oracle and central finite differences."""
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


# ------------------------------------------------------------ refinement

@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("name", ["uniform", "mcf", "mcf_panels"])
def test_fp32_refinement_reaches_1e8(Solver, oracle, name, variant):
    if name == "uniform":
        lp = lpgen.make("uniform_m500_n1k")
    else:
        lp = lpgen.multicommodity(nodes=1500, arcs=6000, commodities=4, seed=2)
    tuning = {"panels_a": 8, "panels_at": 2} if name == "mcf_panels" else None
    ref = oracle.solve(lp, eps_rel=1e-9)
    assert ref.info["status"] == 1
    with Solver.from_lp(lp, tuning=tuning) as s:
        s.configure(eps_rel=1e-8, variant=variant)
        r = s.solve_refined(outer_eps=1e-8, inner_eps=1e-4, max_rounds=8,
                            max_inner_iters=50000)
        for row in s.refine_log():
            print("refine round %d outer %.3e DP %.3g DD %.3g inner iters %d "
                  "status %d inner %.3e t %.2fs cut %d accepted %d" % tuple(row),
                  flush=True)
        assert r["status"] == 1, r
        assert r["rounds"] >= 1
        x, y, z = s.get_iterate()
        inf = s.info()
    # the refined point satisfies the tolerance on the original data,
    # recomputed by the oracle on the CPU
    kk = oracle.kkt(lp, x, y)
    assert kk["maxresid"] <= 1e-8, kk
    assert abs(kk["maxresid"] - r["kkt"]["maxresid"]) <= 1e-12
    assert np.all(x >= 0)
    # error against the optimum p*.  For x >= 0 with residuals r_P, r_D
    # (z = max(0, c - A^T y) >= 0) and an optimal pair (x*, y*):
    #   pobj - p* <= (pobj - dobj) + ||r_D|| ||x*||,  p* - pobj <= ||y*|| ||r_P||
    # (weak duality with z^T x* >= 0 and z*^T x >= 0).  The oracle's 1e-9
    # solution stands in for p*, x* and y*, with its own bound added.
    def bound(k):
        return (abs(k["pobj"] - k["dobj"]) + 1.01 * k["norm_rd"] * np.linalg.norm(ref.x)
                + 1.01 * k["norm_rp"] * np.linalg.norm(ref.y))
    err = abs(kk["pobj"] - ref.kkt["pobj"])
    assert err <= bound(kk) + bound(ref.kkt), (err, bound(kk), bound(ref.kkt))


def test_refinement_cut_rounds_keep_partial_progress(Solver, oracle):
    """Rounds bounded to 3000 inner iterations (the multicommodity LP's
    rounds need up to ~38k): a round cut at its budget keeps the best refined
    point it reached; one that has not improved yet is extended (6000,
    12000, ...); the outer maxresid before each round falls, and the
    refinement still reaches 1e-8, recomputed on the CPU."""
    lp = lpgen.multicommodity(nodes=1500, arcs=6000, commodities=4, seed=2)
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-8, variant=1)
        r = s.solve_refined(outer_eps=1e-8, inner_eps=1e-4, max_rounds=60,
                            max_inner_iters=3000)
        log = s.refine_log()
        for row in log:
            print("refine round %d outer %.3e DP %.3g DD %.3g inner iters %d "
                  "status %d inner %.3e t %.2fs cut %d accepted %d" % tuple(row),
                  flush=True)
        x, y, _ = s.get_iterate()
    assert r["status"] == 1, r
    cut = log[log[:, 5] == 2]                  # rounds ended at their budget
    assert len(cut) >= 1
    assert set(cut[:, 4].astype(int)) <= {3000 << k for k in range(5)}
    assert np.all(cut[:, 9] == 1)              # ... whose progress was kept
    assert np.all(log[:, 9] == 1)              # every round improved the point
    assert np.all(np.diff(log[:, 1]) < 0)
    kk = oracle.kkt(lp, x, y)
    assert kk["maxresid"] <= 1e-8


def test_refinement_stall_window_cuts_rounds_and_keeps_best(Solver, oracle):
    """A stall window of 64 iterations ends a round once its refined point
    has not improved for max(64, 4 x the iterations to its best).  Rounds
    ended that way keep their best point; a round that cannot improve even
    with its window doubled four times ends the refinement with ITER_LIMIT,
    keeping the point before it.  A fresh PDHG solve of a correction LP can
    take thousands of iterations to gain, so such a short window may stop
    short of the target where no window converges."""
    lp = lpgen.multicommodity(nodes=1500, arcs=6000, commodities=4, seed=2)

    def run(stall):
        with Solver.from_lp(lp) as s:
            s.configure(eps_rel=1e-8, variant=1)
            r = s.solve_refined(outer_eps=1e-8, max_rounds=60, max_inner_iters=200000,
                                stall_iters=stall)
            log = s.refine_log()
            x, y, _ = s.get_iterate()
        for row in log:
            print("stall %d refine round %d outer %.3e DP %.3g DD %.3g inner iters %d "
                  "status %d inner %.3e t %.2fs cut %d accepted %d" % ((stall,) + tuple(row)),
                  flush=True)
        return r, log, oracle.kkt(lp, x, y)

    r, log, kk = run(64)
    assert r["status"] in (1, 2), r
    cut = log[:, 8] == 1
    assert cut.any()
    # a cut is recorded as ITER_LIMIT with the stall flag set
    assert np.all(log[cut][:, 5] == 2)
    # every accepted round improved the point the next round starts from
    acc = log[:, 9] == 1
    assert np.all(acc[:-1])
    assert np.all(np.diff(log[:, 1]) < 0)
    if r["status"] == 2:
        # the last round could not improve: the point before it is kept
        assert not acc[-1]
        assert r["kkt"]["maxresid"] == log[-1, 1]
    else:
        assert r["kkt"]["maxresid"] <= 1e-8
    assert abs(kk["maxresid"] - r["kkt"]["maxresid"]) <= 1e-12 + 1e-9 * r["kkt"]["maxresid"]

    # without a stall window the same refinement converges, no round cut
    r, log, kk = run(-1)
    assert r["status"] == 1, r
    assert not (log[:, 8] == 1).any()
    assert kk["maxresid"] <= 1e-8


@pytest.mark.parametrize("inner", [1, 0])
def test_refinement_with_lower_bounds(Solver, oracle, inner):
    # x >= l with l < 0: the correction LP's bound is Delta_P (l - x) and the
    # refined x is clipped at l; FP32 and FP64 inner solves
    lp = lpgen.planted_uniform(m=800, n=2500, k=6, seed=12)
    l = -np.random.default_rng(12).uniform(0.0, 0.5, lp.n)
    ref = oracle.solve(lp, l=l, eps_rel=1e-9)
    assert ref.info["status"] == 1
    with Solver.from_lp(lp, lb=l) as s:
        s.configure(eps_rel=1e-8)
        r = s.solve_refined(outer_eps=1e-8, inner_precision=inner,
                            max_inner_iters=50000)
        for row in s.refine_log():
            print("refine round %d outer %.3e DP %.3g DD %.3g inner iters %d "
                  "status %d inner %.3e t %.2fs cut %d accepted %d" % tuple(row),
                  flush=True)
        assert r["status"] == 1, r
        x, y, _ = s.get_iterate()
    kk = oracle.kkt(lp, x, y, l=l)
    assert kk["maxresid"] <= 1e-8, kk
    assert abs(kk["maxresid"] - r["kkt"]["maxresid"]) <= 1e-12
    # x = D_c (x~), x~ >= l / D_c: the unscaled bound holds to rounding
    assert np.all(x >= l - 4 * np.spacing(np.abs(l)))


@pytest.mark.parametrize("literal", [0, 1])
def test_refinement_snapshots_of_refined_iterate(Solver, oracle, literal):
    # the configured levels apply to the refined iterate; every snapshot
    # satisfies its level on the original data, recomputed on the CPU
    import threading
    lp = lpgen.make("uniform_m500_n1k")
    levels = [1e-2, 1e-4, 1e-6, 1e-8]
    seen, got, ev = [], {}, threading.Event()

    def cb(idx, info, x, y, z):
        # the refinement adds host slots as it reaches levels while earlier
        # callbacks may still run: each call gets its own snapshot's copy
        seen.append((idx, info["level"]))
        got[idx] = (x, y, z)
        if len(seen) == len(levels):
            ev.set()

    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-8, levels=levels, literal_snapshots=literal)
        s.set_snapshot_callback(cb, with_vectors=True)
        r = s.solve_refined(outer_eps=1e-8)
        assert r["status"] == 1
        # one level per measurement when literal, so not all may fire
        cnt = s.snapshot_count()
        assert 1 <= cnt <= len(levels)
        if not literal:
            assert cnt == len(levels)
            assert ev.wait(10)
            assert sorted(seen) == list(enumerate(levels))
        iters = []
        for i in range(cnt):
            info, x, y, z = s.snapshot(i)
            if i in got:
                assert all(np.array_equal(a, b) for a, b in zip(got[i], (x, y, z)))
            assert info["level"] == levels[i]
            kk = oracle.kkt(lp, x, y, want_z=True)
            assert kk["maxresid"] <= info["level"]
            assert abs(kk["maxresid"] - info["maxresid"]) <= 1e-12
            assert np.allclose(z, kk["z"], rtol=1e-12, atol=1e-12)
            iters.append(info["iter"])
        assert iters == sorted(iters)
        assert iters[-1] <= r["inner_iters"]


def test_fp32_bulk_solve_reaches_fp32_accuracy(Solver, oracle):
    lp = lpgen.make("uniform_m500_n1k")
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-5, precision=1)
        st = s.solve(200000)
        assert st == 1
        x, y, _ = s.get_iterate()
    assert oracle.kkt(lp, x, y)["maxresid"] <= 1e-5


# ------------------------------------------------------------ adjoint

def _adjoint_setup(oracle, lp, ruiz=10):
    dr, dc, vs = oracle.ruiz(lp, ruiz)
    eta = 0.9 / oracle.power(lp, vs)
    return dr, dc, eta


@pytest.mark.parametrize("panels", [False, True])
def test_unrolled_matches_oracle_reverse_pass(Solver, oracle, panels):
    lp = lpgen.planted_uniform(m=300, n=700, k=5, seed=41)
    dr, dc, eta = _adjoint_setup(oracle, lp)
    K = 60
    xt = lpgen.target_vector(lp.n, 41)
    xK_or, L_or, gc_or, gb_or, gA_or = oracle.unrolled(lp, dr, dc, eta, eta, K, xt)
    tuning = {"panels_a": 2, "panels_at": 4} if panels else None
    with Solver.from_lp(lp, tuning=tuning) as s:
        s.configure(ruiz_passes=10, power_iters=5)
        grads = {}
        for ck in (1, 7, K):
            xK, tape = s.unrolled_forward(K, ck, eta, eta)
            assert rel(xK, xK_or) <= 1e-12
            gxK = 2 * (xK - xt)
            grads[ck] = tape.backward(gxK)
            tape.free()
    for ck in (1, 7):                    # checkpointing is bitwise invisible
        for a, b in zip(grads[ck], grads[K]):
            assert np.array_equal(a, b)
    gc, gb, gA = grads[K]
    assert rel(gc, gc_or) <= 1e-9 and rel(gb, gb_or) <= 1e-9 and rel(gA, gA_or) <= 1e-9


def test_unrolled_fp32_within_gate(Solver, oracle):
    lp = lpgen.planted_uniform(m=300, n=700, k=5, seed=42)
    dr, dc, eta = _adjoint_setup(oracle, lp)
    K = 60
    xt = lpgen.target_vector(lp.n, 42)
    _, _, gc_or, gb_or, gA_or = oracle.unrolled(lp, dr, dc, eta, eta, K, xt)
    with Solver.from_lp(lp) as s:
        s.configure(ruiz_passes=10, power_iters=5)
        xK, tape = s.unrolled_forward(K, 20, eta, eta, precision=1)
        gc, gb, gA = tape.backward(2 * (xK - xt))
    assert rel(gc, gc_or) <= 1e-3 and rel(gb, gb_or) <= 1e-3 and rel(gA, gA_or) <= 1e-3


@pytest.mark.timeout(900)
def test_adjoint_full_size_vs_oracle_and_fd(Solver, oracle):
    """The adjoint workload at full size: m=50k, n=100k, 8 nonzeros per
    column, K=200 steps, checkpoint every 20, loss ||x_K - x_t||^2."""
    import torch
    from paper_2510_24429_amd.autograd import PDHGUnroll
    lp = lpgen.make("uniform_m50k_n100k_k8")
    dr, dc, eta = _adjoint_setup(oracle, lp)
    K, ck, h = 200, 20, 1e-6
    xt = lpgen.target_vector(lp.n, 3)
    xK_or, L_or, gc_or, gb_or, gA_or = oracle.unrolled(lp, dr, dc, eta, eta, K, xt)
    s = Solver.from_lp(lp)
    s.configure(ruiz_passes=10, power_iters=5)
    dev = torch.device("cuda:0")
    c = torch.tensor(lp.c, device=dev, requires_grad=True)
    b = torch.tensor(lp.b, device=dev, requires_grad=True)
    av = torch.tensor(lp.a_v, device=dev, requires_grad=True)
    xK = PDHGUnroll.apply(c, b, av, s, K, ck, eta, eta)
    loss = ((xK - torch.tensor(xt, device=dev)) ** 2).sum()
    loss.backward()
    gc, gb, gA = (t.grad.cpu().numpy() for t in (c, b, av))
    assert rel(xK.detach().cpu().numpy(), xK_or) <= 1e-12
    assert abs(loss.item() - L_or) <= 1e-10 * L_or
    assert rel(gc, gc_or) <= 1e-9 and rel(gb, gb_or) <= 1e-9 and rel(gA, gA_or) <= 1e-9

    # central differences on 64 random coordinates per group; the loss
    # difference is formed elementwise (sum (x+ - x-)(x+ + x- - 2 t) / 2h).
    # A coordinate whose +-h runs flip a projection mask sits at a kink of
    # the piecewise-linear map: it is skipped (and redrawn) when the oracle's
    # forward pass confirms the flip
    _, h0 = oracle.unrolled_fwd(lp, dr, dc, eta, eta, K)
    rng = np.random.default_rng(7)

    def fwd_gpu(cv, bv, vv):
        s.set_values(vv)
        s.set_rhs_obj(bv, cv)
        x, tape = s.unrolled_forward(K, K, eta, eta)
        tape.free()
        return x

    # Gate: the relative l2 error of the 64 sampled coordinates of each group
    # <= 1e-6, and every coordinate within 1e-4.  A single coordinate cannot
    # be held to 1e-6: each 200-step forward carries ~1e-14 absolute rounding
    # noise per entry, and the elementwise difference sums it over n entries
    # and divides by 2h, a noise floor of ~1e-6 absolute.
    vals = {"c": lp.c, "b": lp.b, "A": lp.a_v}
    for group, g, size in (("c", gc, lp.n), ("b", gb, lp.m), ("A", gA, lp.nnz)):
        done, errs, tries, kinks = 0, [], 0, 0
        fds, gs = [], []
        while done < 64 and tries < 200:
            tries += 1
            t = int(rng.integers(size))
            p = {k: v.copy() for k, v in vals.items()}
            q = {k: v.copy() for k, v in vals.items()}
            p[group][t] += h
            q[group][t] -= h
            xp = fwd_gpu(p["c"], p["b"], p["A"])
            xm = fwd_gpu(q["c"], q["b"], q["A"])
            fd = np.sum((xp - xm) * (xp + xm - 2 * xt)) / (2 * h)
            scale = max(abs(g[t]), 1e-3 * np.max(np.abs(g)))
            err = abs(fd - g[t]) / scale
            if err > 1e-6:
                kw = {"c": "c", "b": "b", "A": "vals"}[group]
                _, hp = oracle.unrolled_fwd(lp, dr, dc, eta, eta, K, **{kw: p[group]})
                _, hm = oracle.unrolled_fwd(lp, dr, dc, eta, eta, K, **{kw: q[group]})
                if hp != h0 or hm != h0:
                    kinks += 1
                    continue
            errs.append(err)
            fds.append(fd)
            gs.append(g[t])
            done += 1
        assert done == 64, (group, done, kinks)
        l2 = np.linalg.norm(np.array(fds) - np.array(gs)) / np.linalg.norm(gs)
        print(f"FD {group}: 64 coords, l2 rel {l2:.2e}, max coord rel "
              f"{max(errs):.2e}, kinks skipped {kinks}", flush=True)
        assert l2 <= 1e-6, (group, l2)
        assert max(errs) <= 1e-4, (group, max(errs))
    fwd_gpu(lp.c, lp.b, lp.a_v)
    s.close()


def test_tape_outliving_its_solver_is_released_cleanly(Solver, oracle):
    # regression: a tape freed after its context was destroyed must not touch
    # the destroyed context
    from paper_2510_24429_amd._lib import PDHGError
    lp = lpgen.planted_uniform(m=100, n=200, k=4, seed=43)
    s = Solver.from_lp(lp)
    s.configure(ruiz_passes=10, power_iters=5)
    xK, tape = s.unrolled_forward(10, 5, 0.1, 0.1)
    s.close()
    with pytest.raises(PDHGError):
        tape.backward(np.ones(lp.n))
    tape.free()


def test_stale_tape_is_refused(Solver):
    """A tape replays the context's current problem data: after a change of
    values, right-hand side or objective, scaling or problem, its backward
    pass is refused instead of mixing two problems."""
    from paper_2510_24429_amd._lib import PDHGError
    lp = lpgen.planted_uniform(m=100, n=200, k=4, seed=44)
    other = lpgen.planted_uniform(m=60, n=150, k=3, seed=45)
    g = np.linspace(-1.0, 1.0, lp.n)
    with Solver.from_lp(lp) as s:
        s.configure(ruiz_passes=10, power_iters=5)
        _, tape = s.unrolled_forward(10, 5, 0.1, 0.1)
        ref = tape.backward(g)
        again = tape.backward(g)            # unchanged data: same result
        for a, b in zip(ref, again):
            assert np.array_equal(a, b)
        tape.free()
        changes = [lambda: s.set_values(lp.a_v * 1.5),
                   lambda: s.set_rhs_obj(c=lp.c * 2.0),
                   lambda: s.configure(ruiz_passes=10, power_iters=5)]
        for change in changes:
            s.set_values(lp.a_v)
            s.set_rhs_obj(lp.b, lp.c)
            s.configure(ruiz_passes=10, power_iters=5)
            _, tape = s.unrolled_forward(10, 5, 0.1, 0.1)
            change()
            with pytest.raises(PDHGError, match="STATE"):
                tape.backward(g)
            tape.free()
        # a reload with other sizes frees the tape's memory; the handle is
        # refused and still released cleanly
        s.set_values(lp.a_v)
        s.set_rhs_obj(lp.b, lp.c)
        s.configure(ruiz_passes=10, power_iters=5)
        _, tape = s.unrolled_forward(10, 5, 0.1, 0.1)
        s.load_lp(other)
        with pytest.raises(PDHGError, match="STATE"):
            tape.backward(np.ones(other.n))
        tape.free()
        # the reloaded context runs a fresh forward and backward
        s.configure(ruiz_passes=10, power_iters=5)
        _, tape = s.unrolled_forward(10, 5, 0.1, 0.1)
        gc, gb, gA = tape.backward(np.ones(other.n))
        assert gc.shape == (other.n,) and gb.shape == (other.m,)
        assert np.isfinite(gA).all()
        tape.free()
