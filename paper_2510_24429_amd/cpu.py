"""The CPU platform (no GPU): the restarted PDHG on the host's cores
(pdhg_cpu_*), the plain step pair (pdhg_cpu_steps) and the host's streaming
read bandwidth (pdhg_cpu_stream_bw).  Argument marshalling only."""
import ctypes as C

import numpy as np

from . import _lib as L


def _arr(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, ctx=None):
    if rc < 0:
        msg = ""
        if ctx:
            m = L.lib().pdhg_cpu_last_error(ctx)
            msg = m.decode() if m else ""
        raise L.PDHGError(rc, msg)
    return rc


class CpuSolver:
    """Restarted PDHG on `threads` host threads for min c^T x, Ax = b,
    x >= lb, FP64 (the GPU Solver's method and decisions)."""

    def __init__(self, m, n, a_rp, a_ci, a_v, at_rp, at_ci, at_v, b, c,
                 lb=None, threads: int = 1):
        self.lib = L.lib()
        ctx = C.c_void_p()
        _check(self.lib.pdhg_cpu_create(int(threads), C.byref(ctx)))
        self.ctx = ctx
        self.m, self.n, self.nnz = int(m), int(n), int(len(a_v))
        self.threads = int(threads)
        self._keep = None
        arrs = [_arr(a_rp, np.int64), _arr(a_ci, np.int32), _arr(a_v, np.float64),
                _arr(at_rp, np.int64), _arr(at_ci, np.int32), _arr(at_v, np.float64),
                _arr(b, np.float64), _arr(c, np.float64),
                None if lb is None else _arr(lb, np.float64)]
        _check(self.lib.pdhg_cpu_load(self.ctx, self.m, self.n, self.nnz,
                                      *[_p(a) for a in arrs]), self.ctx)

    @classmethod
    def from_lp(cls, lp, lb=None, threads: int = 1) -> "CpuSolver":
        return cls(lp.m, lp.n, lp.a_rp, lp.a_ci, lp.a_v, lp.at_rp, lp.at_ci,
                   lp.at_v, lp.b, lp.c, lb=lb, threads=threads)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pdhg_cpu_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_threads(self, threads: int):
        _check(self.lib.pdhg_cpu_set_threads(self.ctx, int(threads)), self.ctx)
        self.threads = int(threads)

    def configure(self, **params):
        p, keep = L.default_params(**params)
        self._keep = keep
        _check(self.lib.pdhg_cpu_configure(self.ctx, C.byref(p)), self.ctx)
        return self

    def iterate(self, max_iters: int) -> int:
        st = C.c_int(0)
        _check(self.lib.pdhg_cpu_iterate(self.ctx, int(max_iters), C.byref(st)), self.ctx)
        return st.value

    def solve(self, max_iters: int = 2 ** 62) -> int:
        return self.iterate(max_iters)

    def cancel(self):
        _check(self.lib.pdhg_cpu_cancel(self.ctx), self.ctx)

    def info(self) -> dict:
        o = L.Info()
        _check(self.lib.pdhg_cpu_get_info(self.ctx, C.byref(o)), self.ctx)
        return o.asdict()

    def get_iterate(self):
        x, y, z = np.empty(self.n), np.empty(self.m), np.empty(self.n)
        _check(self.lib.pdhg_cpu_get_iterate(self.ctx, _p(x), _p(y), _p(z)), self.ctx)
        return x, y, z

    def get_scaling(self):
        dr, dc = np.empty(self.m), np.empty(self.n)
        _check(self.lib.pdhg_cpu_get_scaling(self.ctx, _p(dr), _p(dc)), self.ctx)
        return dr, dc

    def eval_log(self, cap: int = 4096) -> np.ndarray:
        out = np.zeros(cap * 8)
        cnt = C.c_int(0)
        _check(self.lib.pdhg_cpu_eval_log(self.ctx, _p(out), cap, C.byref(cnt)), self.ctx)
        return out.reshape(-1, 8)[:min(cnt.value, cap)]

    def snapshot_count(self) -> int:
        cnt = C.c_int(0)
        _check(self.lib.pdhg_cpu_snapshot_count(self.ctx, C.byref(cnt)), self.ctx)
        return cnt.value

    def snapshot(self, idx: int):
        info = L.SnapInfo()
        x, y, z = np.empty(self.n), np.empty(self.m), np.empty(self.n)
        _check(self.lib.pdhg_cpu_snapshot(self.ctx, idx, C.byref(info), _p(x),
                                          _p(y), _p(z)), self.ctx)
        return info.asdict(), x, y, z


def stream_bandwidth(threads: int, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Host streaming read bandwidth (GB/s) with `threads` threads."""
    g = C.c_double(0.0)
    _check(L.lib().pdhg_cpu_stream_bw(int(threads), int(nbytes), int(reps), C.byref(g)))
    return g.value


def cpu_steps(lp, x, y, tau: float, sigma: float, K: int, threads: int,
              vals=None, b=None, c=None):
    """K plain steps of the LP's CSR pair (or of the values `vals` in A's
    order, scattered into A^T through the transpose permutation) from x, y
    (copied).  Returns (x_K, y_K, seconds)."""
    a_v = _arr(lp.a_v if vals is None else vals, np.float64)
    at_v = _arr(lp.at_v, np.float64)
    if vals is not None:
        at_v = np.empty_like(at_v)
        at_v[lp.a_perm_to_at()] = a_v
    x = _arr(x, np.float64).copy()
    y = _arr(y, np.float64).copy()
    bb = _arr(lp.b if b is None else b, np.float64)
    cc = _arr(lp.c if c is None else c, np.float64)
    a_rp, a_ci = _arr(lp.a_rp, np.int64), _arr(lp.a_ci, np.int32)
    at_rp, at_ci = _arr(lp.at_rp, np.int64), _arr(lp.at_ci, np.int32)
    secs = C.c_double(0.0)
    rc = L.lib().pdhg_cpu_steps(lp.m, lp.n, _p(a_rp), _p(a_ci), _p(a_v), _p(at_rp),
                                _p(at_ci), _p(at_v), _p(bb), _p(cc), tau, sigma,
                                int(K), int(threads), _p(x), _p(y), C.byref(secs))
    L.check(rc)
    return x, y, secs.value
