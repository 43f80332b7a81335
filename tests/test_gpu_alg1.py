"""Algorithm 1 (Section 3.1) concurrent crossover harness on the GPU, with a
stand-in crossover routine (the simplex crossover itself is external)."""
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


def test_first_successful_crossover_wins_and_cancels(Solver, oracle):
    lp = lpgen.planted_uniform(m=20000, n=60000, k=5, seed=4)
    levels = oracle.alg1_levels(1e-2, 1e-10)
    calls, lock = [], threading.Lock()

    def crossover(idx, info, x, y, z, cancelled):
        # stand-in: a start looser than 1e-4 never finishes (it runs until it
        # is cancelled); one at 1e-4 or tighter finishes after 50 ms
        with lock:
            calls.append((idx, info["level"], info["maxresid"]))
        assert np.all(z >= 0) and x.shape == (lp.n,) and y.shape == (lp.m,)
        if info["level"] > 1e-4:
            while not cancelled():
                time.sleep(0.005)
            return False
        time.sleep(0.05)
        return True

    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-10, levels=levels)
        t0 = time.time()
        winner, status = s.concurrent_crossover(crossover)
        dt = time.time() - t0
        info = s.info()
        snaps = [s.snapshot(i)[0] for i in range(s.snapshot_count())]
    assert status == 4                          # PDHG stopped by the winner
    assert snaps[winner]["level"] == 1e-4
    assert info["kkt"]["maxresid"] > 1e-10      # it never reached eps_rel
    assert sorted(c[1] for c in calls)[-1] == 1e-2   # earlier starts launched
    assert all(c[2] <= c[1] for c in calls)
    assert dt < 60


def test_no_winner_runs_final_crossover_on_converged_iterate(Solver, oracle):
    lp = lpgen.make("uniform_m500_n1k")
    seen = []

    def crossover(idx, info, x, y, z, cancelled):
        seen.append((idx, info["level"]))
        if idx == -1:
            kk = oracle.kkt(lp, x.copy(), y.copy())
            assert kk["maxresid"] <= 1e-6
        return False

    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-6, levels=[1e-2, 1e-4])     # eps_rel not a level
        winner, status = s.concurrent_crossover(crossover, max_threads=1)
    assert winner == -2 and status == 1
    assert sorted(seen)[0] == (-1, 1e-6)
    assert sorted(l for i, l in seen if i >= 0) == [1e-4, 1e-2]


def test_refined_harness_launches_from_refined_snapshots(Solver, oracle):
    # Algorithm 1 over FP32 + refinement: the refined iterate's snapshots
    # start the crossovers; the first that succeeds stops the refinement
    lp = lpgen.planted_powerlaw(m=4000, n=20000, kmax=1000, seed=1)
    levels = oracle.alg1_levels(1e-2, 1e-9)
    calls, lock = [], threading.Lock()

    def crossover(idx, info, x, y, z, cancelled):
        with lock:
            calls.append((idx, info["level"], info["maxresid"]))
        kk = oracle.kkt(lp, x.copy(), y.copy())
        ok.append(kk["maxresid"] <= info["level"])
        if info["level"] > 1e-3:
            while not cancelled():
                time.sleep(0.005)
            return False
        return True

    ok = []
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-9, levels=levels)
        winner, status, info = s.concurrent_crossover_refined(crossover)
        snaps = [s.snapshot(i)[0] for i in range(s.snapshot_count())]
    assert winner >= 0 and snaps[winner]["level"] <= 1e-3
    # the winner's cancel stops the refinement at its next check; a round
    # already under way may still finish it first
    assert status in (1, 4) and info["status"] == status
    assert all(ok) and all(c[2] <= c[1] for c in calls)
    assert min(c[1] for c in calls) >= 1e-9


def test_refined_harness_without_winner_runs_final_crossover(Solver, oracle):
    lp = lpgen.make("uniform_m500_n1k")
    seen = []

    def crossover(idx, info, x, y, z, cancelled):
        seen.append((idx, info["level"]))
        return False

    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-8, levels=[1e-2, 1e-4])
        winner, status, info = s.concurrent_crossover_refined(crossover, max_threads=1)
        x, y, _ = s.get_iterate()
    assert winner == -2 and status == 1 and info["status"] == 1
    assert (-1, 1e-8) in seen
    assert sorted(l for i, l in seen if i >= 0) == [1e-4, 1e-2]
    assert oracle.kkt(lp, x, y)["maxresid"] <= 1e-8


def test_busy_threads_do_not_hold_up_pdhg(Solver):
    """With one crossover thread and slow crossovers, later snapshots queue
    and PDHG keeps iterating (Algorithm 1's loop runs while its threads do):
    the solve's own time stays far below the crossovers' total, and every
    snapshot still gets its crossover, one at a time."""
    lp = lpgen.make("uniform_m500_n1k")
    levels = [1e-2, 1e-3, 1e-4, 1e-5]
    starts, lock = [], threading.Lock()
    active = [0]

    def crossover(idx, info, x, y, z, cancelled):
        with lock:
            active[0] += 1
            starts.append((idx, active[0]))
        time.sleep(0.4)
        with lock:
            active[0] -= 1
        return False

    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-6, levels=levels)
        t0 = time.time()
        winner, status = s.concurrent_crossover(crossover, max_threads=1)
        dt = time.time() - t0
        t_iter = s.info()["t_iter"]
    assert winner == -2 and status == 1
    assert sorted(i for i, _ in starts if i >= 0) == [0, 1, 2, 3]
    # the thread limit holds for the snapshot crossovers; the final one runs
    # on the calling thread beside them
    assert all(a <= 2 for _, a in starts)
    assert dt >= 4 * 0.4
    assert t_iter < 0.8, t_iter


def test_outside_cancel_reaches_the_crossovers(Solver):
    """pdhg_cancel from another thread during the harness stops PDHG and sets
    the crossovers' cancel word: a crossover that waits for it returns, and
    the call ends with PDHG_CANCELLED and no winner."""
    lp = lpgen.planted_uniform(m=20000, n=60000, k=5, seed=4)
    started, saw = threading.Event(), []

    def crossover(idx, info, x, y, z, cancelled):
        started.set()
        t0 = time.time()
        while not cancelled() and time.time() - t0 < 30:
            time.sleep(0.005)
        saw.append(cancelled())
        return False

    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-12, levels=[1e-2], max_iters=2_000_000)

        def cancel_once_started():
            if started.wait(30):
                s.cancel()

        th = threading.Thread(target=cancel_once_started)
        th.start()
        t0 = time.time()
        winner, status = s.concurrent_crossover(crossover)
        dt = time.time() - t0
        th.join()
    assert status == 4 and winner == -2
    assert saw == [True]
    assert dt < 30


def test_cancel_before_the_call_is_dropped(Solver):
    """A cancel requested before the harness starts does not stop it."""
    lp = lpgen.make("uniform_m500_n1k")
    with Solver.from_lp(lp) as s:
        s.configure(eps_rel=1e-6, levels=[1e-4])
        s.cancel()
        winner, status = s.concurrent_crossover(lambda *a: False)
        assert status == 1 and winner == -2
        s.configure(eps_rel=1e-6, levels=[1e-4])
        s.cancel()
        winner, status, info = s.concurrent_crossover_refined(lambda *a: False)
        assert status == 1 and winner == -2 and info["status"] == 1
