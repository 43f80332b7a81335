"""The CPU platform's plain PDHG steps (host only): against the oracle's
plain steps, and invariant in the thread count."""
import numpy as np
import pytest

from paper_2510_24429_amd import lpgen
from paper_2510_24429_amd.cpu import cpu_steps


def _scaled(oracle, lp):
    dr, dc, vs = oracle.ruiz(lp, 10)
    eta = 0.9 / oracle.power(lp, vs)
    return dr, dc, vs, eta


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_cpu_steps_match_oracle_plain_steps(oracle, threads):
    lp = lpgen.planted_powerlaw(m=2000, n=9000, kmax=900, seed=5)
    dr, dc, vs, eta = _scaled(oracle, lp)
    K = 40
    xK_or, _ = oracle.unrolled_fwd(lp, dr, dc, eta, eta, K)
    x, y, secs = cpu_steps(lp, np.zeros(lp.n), np.zeros(lp.m), eta, eta, K,
                           threads, vals=vs, b=dr * lp.b, c=dc * lp.c)
    xK = dc * x
    assert np.linalg.norm(xK - xK_or) <= 1e-12 * np.linalg.norm(xK_or)
    assert secs > 0


def test_cpu_steps_bitwise_across_thread_counts():
    lp = lpgen.make("uniform_m500_n1k")
    out = [cpu_steps(lp, np.zeros(lp.n), np.zeros(lp.m), 0.05, 0.05, 30, t)
           for t in (1, 2, 7)]
    for x, y, _ in out[1:]:
        assert np.array_equal(x, out[0][0]) and np.array_equal(y, out[0][1])


def test_cpu_steps_reject_bad_arguments():
    from paper_2510_24429_amd import _lib as L
    lp = lpgen.make("uniform_m500_n1k")
    with pytest.raises(L.PDHGError):
        cpu_steps(lp, np.zeros(lp.n), np.zeros(lp.m), 0.1, 0.1, 3, 0)
