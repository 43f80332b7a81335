"""pdhg_spmv_noalloc, the allocation-free SpMV, against pdhg_spmv through the
C ABI: the same kernels, so the products must agree bitwise, on two loaded
problems in a row (the second smaller), in both precisions and on both the
scaled and the loaded values, with column panels (partial sums) in use.
Sizes beyond the fixed device scratch are rejected with an error and run no
kernel."""
import numpy as np
import pytest

from paper_2510_24429_amd import _lib as L
from paper_2510_24429_amd import lpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def _products(s, torch, tag):
    """Every (which, scaled, precision) product by both entry points, the
    no-alloc one writing into preallocated device tensors; checks that the
    device's free memory does not move across the no-alloc calls."""
    dev = f"cuda:{s.device}"
    rng = np.random.default_rng(5)
    vecs = {0: torch.tensor(rng.standard_normal(s.n), device=dev),
            1: torch.tensor(rng.standard_normal(s.m), device=dev)}
    outs = {0: torch.empty(s.m, dtype=torch.float64, device=dev),
            1: torch.empty(s.n, dtype=torch.float64, device=dev)}
    cases = [(w, sc, p) for w in (0, 1) for sc in (False, True)
             for p in (L.FP64, L.FP32)]
    # the allocating entry point first: it also runs every kernel once
    ref = {c: s.spmv(c[0], vecs[c[0]], scaled=c[1], precision=c[2]).cpu().numpy()
           for c in cases}
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(s.device)[0]
    got = {}
    for c in cases:
        s.spmv_noalloc(c[0], vecs[c[0]], scaled=c[1], precision=c[2],
                       out=outs[c[0]])
        got[c] = outs[c[0]].cpu().numpy()
    free1 = torch.cuda.mem_get_info(s.device)[0]
    print(f"[no_alloc] {tag}: m={s.m} n={s.n} free before {free0} after {free1}",
          flush=True)
    assert free1 == free0, (free0, free1)
    for c in cases:
        assert np.array_equal(got[c], ref[c]), (tag, c)
        assert np.isfinite(got[c]).all()
    # host arrays in and out, once per side
    for w in (0, 1):
        h = vecs[w].cpu().numpy()
        assert np.array_equal(s.spmv_noalloc(w, h, scaled=True), ref[(w, True, L.FP64)])


def test_noalloc_matches_spmv_on_two_problems(torch):
    from paper_2510_24429_amd.solver import Solver
    big = lpgen.planted_powerlaw(m=20_000, n=100_000, kmax=3000, seed=11)
    small = lpgen.make("uniform_m500_n1k")
    print("[no_alloc] first problem: power-law 20k x 100k, panels 4 / 2", flush=True)
    with Solver.from_lp(big, tuning={"panels_a": 4, "panels_at": 2}) as s:
        assert (s.panel_count(0), s.panel_count(1)) == (4, 2)
        s.configure(eps_rel=1e-6)
        _products(s, torch, "power-law 20k x 100k")
    print("[no_alloc] second problem: uniform 500 x 1k", flush=True)
    with Solver.from_lp(small) as s:
        s.configure(eps_rel=1e-6)
        _products(s, torch, "uniform 500 x 1k")


def test_noalloc_limit(torch):
    """One row over 6M columns: FP64 staging (8 (rows + cols) bytes) fits the
    64 MiB scratch and matches pdhg_spmv; FP32 staging (12 bytes per entry)
    does not and is refused before any kernel runs."""
    from paper_2510_24429_amd.solver import Solver
    assert L.SPMV_NOALLOC_MAX_BYTES == 64 << 20
    n = 6_000_000
    rows = np.zeros(n, dtype=np.int64)
    cols = np.arange(n, dtype=np.int64)
    vals = np.where(cols % 3 == 0, 1.0, -2.0)
    lp = lpgen.from_coo(1, n, rows, cols, vals, np.ones(1), np.ones(n), name="wide")
    print("[no_alloc] limit: 1 x 6M", flush=True)
    with Solver.from_lp(lp) as s:
        x = np.random.default_rng(2).integers(-4, 5, n).astype(np.float64)
        ref = s.spmv(0, x)
        assert np.array_equal(s.spmv_noalloc(0, x), ref)
        assert ref[0] == float(vals @ x)
        with pytest.raises(RuntimeError, match="scratch"):
            s.spmv_noalloc(0, x, precision=L.FP32)
        # the context is still usable after the refusal
        assert np.array_equal(s.spmv_noalloc(0, x), ref)
