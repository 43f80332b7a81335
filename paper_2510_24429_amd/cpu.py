"""The CPU platform: plain PDHG steps on the host's cores (no GPU)."""
import ctypes as C

import numpy as np

from . import _lib as L


def cpu_steps(lp, x, y, tau: float, sigma: float, K: int, threads: int,
              vals=None, b=None, c=None):
    """K plain steps of the LP's CSR pair (or of the values `vals` in A's
    order, scattered into A^T through the transpose permutation) from x, y
    (copied).  Returns (x_K, y_K, seconds)."""
    def arr(a, dt):
        return np.ascontiguousarray(a, dtype=dt)
    a_v = arr(lp.a_v if vals is None else vals, np.float64)
    at_v = arr(lp.at_v, np.float64)
    if vals is not None:
        at_v = np.empty_like(at_v)
        at_v[lp.a_perm_to_at()] = a_v
    x = arr(x, np.float64).copy()
    y = arr(y, np.float64).copy()
    bb = arr(lp.b if b is None else b, np.float64)
    cc = arr(lp.c if c is None else c, np.float64)
    a_rp, a_ci = arr(lp.a_rp, np.int64), arr(lp.a_ci, np.int32)
    at_rp, at_ci = arr(lp.at_rp, np.int64), arr(lp.at_ci, np.int32)
    secs = C.c_double(0.0)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    rc = L.lib().pdhg_cpu_steps(lp.m, lp.n, p(a_rp), p(a_ci), p(a_v), p(at_rp),
                                p(at_ci), p(at_v), p(bb), p(cc), tau, sigma,
                                int(K), int(threads), p(x), p(y), C.byref(secs))
    L.check(rc)
    return x, y, secs.value
