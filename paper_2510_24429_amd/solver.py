"""Thin Python front end of libpdhg.so.

Inputs may be numpy arrays (host memory) or torch tensors (host or device
memory); outputs are numpy arrays unless ``device=True`` asks for torch
tensors on the context's GPU.  torch supplies device memory and the stream;
all arithmetic runs in the library.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Arg:
    """Pointer + memory kind for one input array (keeps the buffer alive)."""

    def __init__(self, a, dtype, count: int, name: str):
        if a is None:
            self.ptr, self.mem, self.keep = None, L.MEM_HOST, None
            return
        if _is_torch(a):
            torch = _torch()
            tdt = {np.float64: torch.float64, np.int64: torch.int64,
                   np.int32: torch.int32}[dtype]
            t = a.detach()
            if t.dtype != tdt:
                t = t.to(tdt)
            t = t.contiguous()
            if t.numel() != count:
                raise ValueError(f"{name}: expected {count} entries, got {t.numel()}")
            self.keep = t
            self.ptr = C.c_void_p(t.data_ptr())
            self.mem = L.MEM_DEVICE if t.is_cuda else L.MEM_HOST
        else:
            arr = np.ascontiguousarray(np.asarray(a), dtype=dtype)
            if arr.size != count:
                raise ValueError(f"{name}: expected {count} entries, got {arr.size}")
            self.keep = arr
            self.ptr = arr.ctypes.data_as(C.c_void_p)
            self.mem = L.MEM_HOST


def _same_mem(*args):
    mems = {a.mem for a in args if a.ptr is not None}
    if len(mems) > 1:
        raise ValueError("mix of host and device inputs in one call")
    return mems.pop() if mems else L.MEM_HOST


class Solver:
    """Restarted PDHG on one GPU for min c^T x, Ax = b, x >= lb."""

    def __init__(self, m, n, a_rp, a_ci, a_v, at_rp, at_ci, at_v, b, c,
                 lb=None, device: int = 0, use_torch_stream: bool = True,
                 tuning: Optional[dict] = None):
        self.lib = L.lib()
        self.m, self.n = int(m), int(n)
        nnz = int(len(a_v)) if not _is_torch(a_v) else int(a_v.numel())
        self.nnz = nnz
        stream = None
        if use_torch_stream:
            torch = _torch()
            if torch.cuda.is_available():
                torch.cuda.set_device(device)
                stream = C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
        self.device = device
        ctx = C.c_void_p()
        L.check_create(self.lib.pdhg_create(device, stream, C.byref(ctx)))
        self.ctx = ctx
        self._keep = None
        self._cb = None
        self._tapes = []
        for k, v in (tuning or {}).items():
            L.check(self.lib.pdhg_set_tuning(self.ctx, k.encode(), int(v)), self.ctx)
        self.load(m, n, a_rp, a_ci, a_v, at_rp, at_ci, at_v, b, c, lb)

    def load(self, m, n, a_rp, a_ci, a_v, at_rp, at_ci, at_v, b, c, lb=None):
        """pdhg_load: (re)load a problem into this context."""
        m, n = int(m), int(n)
        nnz = int(len(a_v)) if not _is_torch(a_v) else int(a_v.numel())
        args = [_Arg(a_rp, np.int64, m + 1, "a_rp"),
                _Arg(a_ci, np.int32, nnz, "a_ci"),
                _Arg(a_v, np.float64, nnz, "a_v"),
                _Arg(at_rp, np.int64, n + 1, "at_rp"),
                _Arg(at_ci, np.int32, nnz, "at_ci"),
                _Arg(at_v, np.float64, nnz, "at_v"),
                _Arg(b, np.float64, m, "b"),
                _Arg(c, np.float64, n, "c"),
                _Arg(lb, np.float64, n, "lb")]
        mem = _same_mem(*args)
        L.check(self.lib.pdhg_load(self.ctx, m, n, nnz,
                                   *[a.ptr for a in args], mem), self.ctx)
        self.m, self.n, self.nnz = m, n, nnz
        return self

    def load_lp(self, lp, lb=None):
        return self.load(lp.m, lp.n, lp.a_rp, lp.a_ci, lp.a_v, lp.at_rp,
                         lp.at_ci, lp.at_v, lp.b, lp.c, lb=lb)

    @classmethod
    def from_lp(cls, lp, lb=None, **kw) -> "Solver":
        return cls(lp.m, lp.n, lp.a_rp, lp.a_ci, lp.a_v, lp.at_rp, lp.at_ci,
                   lp.at_v, lp.b, lp.c, lb=lb, **kw)

    def close(self):
        if getattr(self, "ctx", None):
            for ref in getattr(self, "_tapes", []):
                t = ref()
                if t is not None:
                    t.free()
            self._tapes = []
            self.lib.pdhg_destroy(self.ctx)
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

    # ------------------------------------------------------------- setup
    def configure(self, **params):
        p, keep = L.default_params(**params)
        self._keep = keep
        L.check(self.lib.pdhg_configure(self.ctx, C.byref(p)), self.ctx)
        return self

    def set_iterate(self, x=None, y=None):
        ax = _Arg(x, np.float64, self.n, "x")
        ay = _Arg(y, np.float64, self.m, "y")
        L.check(self.lib.pdhg_set_iterate(self.ctx, ax.ptr, ay.ptr,
                                          _same_mem(ax, ay)), self.ctx)

    def set_values(self, a_v):
        a = _Arg(a_v, np.float64, self.nnz, "a_v")
        L.check(self.lib.pdhg_set_values(self.ctx, a.ptr, a.mem), self.ctx)

    def set_rhs_obj(self, b=None, c=None):
        ab = _Arg(b, np.float64, self.m, "b")
        ac = _Arg(c, np.float64, self.n, "c")
        L.check(self.lib.pdhg_set_rhs_obj(self.ctx, ab.ptr, ac.ptr,
                                          _same_mem(ab, ac)), self.ctx)

    def set_tuning(self, key: str, value: int):
        L.check(self.lib.pdhg_set_tuning(self.ctx, key.encode(), int(value)), self.ctx)

    # ------------------------------------------------------------- run
    def iterate(self, max_iters: int) -> int:
        st = C.c_int(0)
        L.check(self.lib.pdhg_iterate(self.ctx, int(max_iters), C.byref(st)), self.ctx)
        return st.value

    def solve(self, max_iters: int = 2 ** 62) -> int:
        return self.iterate(max_iters)

    def cancel(self):
        L.check(self.lib.pdhg_cancel(self.ctx), self.ctx)

    def info(self) -> dict:
        o = L.Info()
        L.check(self.lib.pdhg_get_info(self.ctx, C.byref(o)), self.ctx)
        return o.asdict()

    def residuals(self, which: int = 0) -> dict:
        o = L.KKT()
        L.check(self.lib.pdhg_residuals(self.ctx, which, C.byref(o)), self.ctx)
        return o.asdict()

    def _out(self, count: int, device: bool):
        if device:
            torch = _torch()
            t = torch.empty(count, dtype=torch.float64, device=f"cuda:{self.device}")
            return t, C.c_void_p(t.data_ptr()), L.MEM_DEVICE
        a = np.empty(count)
        return a, a.ctypes.data_as(C.c_void_p), L.MEM_HOST

    def get_iterate(self, device: bool = False):
        x, px, mem = self._out(self.n, device)
        y, py, _ = self._out(self.m, device)
        z, pz, _ = self._out(self.n, device)
        L.check(self.lib.pdhg_get_iterate(self.ctx, px, py, pz, mem), self.ctx)
        return x, y, z

    def get_scaling(self):
        dr, pr, mem = self._out(self.m, False)
        dc, pc, _ = self._out(self.n, False)
        L.check(self.lib.pdhg_get_scaling(self.ctx, pr, pc, mem), self.ctx)
        return dr, dc

    def eval_log(self, cap: int = 4096) -> np.ndarray:
        buf = np.zeros((cap, 8))
        cnt = C.c_int(0)
        L.check(self.lib.pdhg_eval_log(self.ctx, buf.ctypes.data_as(C.c_void_p),
                                       cap, C.byref(cnt)), self.ctx)
        return buf[:min(cnt.value, cap)]

    # ------------------------------------------------------------- snapshots
    def snapshot_count(self) -> int:
        k = C.c_int(0)
        L.check(self.lib.pdhg_snapshot_count(self.ctx, C.byref(k)), self.ctx)
        return k.value

    def snapshot(self, idx: int, device: bool = False):
        inf = L.SnapInfo()
        x, px, mem = self._out(self.n, device)
        y, py, _ = self._out(self.m, device)
        z, pz, _ = self._out(self.n, device)
        L.check(self.lib.pdhg_snapshot(self.ctx, idx, C.byref(inf), px, py, pz, mem),
                self.ctx)
        return inf.asdict(), x, y, z

    def snapshot_info(self, idx: int) -> dict:
        """pdhg_snapshot without the vectors: level, iteration, maxresid and
        wall time of snapshot idx."""
        inf = L.SnapInfo()
        L.check(self.lib.pdhg_snapshot(self.ctx, idx, C.byref(inf), None, None, None,
                                       L.MEM_HOST), self.ctx)
        return inf.asdict()

    def set_snapshot_callback(self, fn, with_vectors: bool = False):
        """fn(idx, info_dict) -- or, with_vectors, fn(idx, info_dict, x, y, z)
        with copies of the snapshot's unscaled vectors -- runs on a library
        thread after the snapshot's host copy."""
        n, m = self.n, self.m

        def _cb(user, idx, info, px, py, pz):
            if with_vectors:
                fn(idx, info.contents.asdict(),
                   np.ctypeslib.as_array(px, shape=(n,)).copy(),
                   np.ctypeslib.as_array(py, shape=(m,)).copy(),
                   np.ctypeslib.as_array(pz, shape=(n,)).copy())
            else:
                fn(idx, info.contents.asdict())
        self._cb = L.SNAP_CB(_cb)
        L.check(self.lib.pdhg_set_snapshot_callback(self.ctx, self._cb, None), self.ctx)

    # ------------------------------------------------------------- Algorithm 1
    def _crossover_fn(self, fn):
        n, m = self.n, self.m

        def _fn(user, idx, info, px, py, pz, pcancel):
            x = np.ctypeslib.as_array(px, shape=(n,))
            y = np.ctypeslib.as_array(py, shape=(m,))
            z = np.ctypeslib.as_array(pz, shape=(n,))
            try:
                ok = fn(idx, info.contents.asdict(), x, y, z,
                        lambda: pcancel[0] != 0)
            except Exception:
                ok = False
            return 1 if ok else 0

        return L.CROSSOVER_FN(_fn)

    def concurrent_crossover(self, fn, max_threads: int = 0,
                             max_iters: int = 2 ** 62):
        """Algorithm 1: fn(idx, info, x, y, z, cancelled) -> bool runs on a
        library thread for every snapshot (idx -1: the converged iterate);
        x, y, z are numpy views valid during the call, cancelled() tells
        whether another call has already won.  Returns (winner, status)."""
        cb = self._crossover_fn(fn)
        win, st = C.c_int(0), C.c_int(0)
        L.check(self.lib.pdhg_concurrent_crossover(self.ctx, cb, None, max_threads,
                                                   int(max_iters), C.byref(win),
                                                   C.byref(st)), self.ctx)
        return win.value, st.value

    def concurrent_crossover_refined(self, fn, max_threads: int = 0, **kw):
        """Algorithm 1 over FP32 bulk iterations with FP64 refinement (keyword
        arguments as for solve_refined).  Returns (winner, status, info)."""
        cb = self._crossover_fn(fn)
        rp = L.RefineParams()
        L.check(self.lib.pdhg_refine_params_default(C.byref(rp)))
        for k, v in kw.items():
            setattr(rp, k, v)
        info = L.RefineInfo()
        win, st = C.c_int(0), C.c_int(0)
        L.check(self.lib.pdhg_concurrent_crossover_refined(
            self.ctx, cb, None, max_threads, C.byref(rp), C.byref(win),
            C.byref(st), C.byref(info)), self.ctx)
        return win.value, st.value, info.asdict()

    # ------------------------------------------------------------- refinement
    def solve_refined(self, **kw) -> dict:
        rp = L.RefineParams()
        L.check(self.lib.pdhg_refine_params_default(C.byref(rp)))
        for k, v in kw.items():
            setattr(rp, k, v)
        info = L.RefineInfo()
        L.check(self.lib.pdhg_solve_refined(self.ctx, C.byref(rp), C.byref(info)),
                self.ctx)
        return info.asdict()

    def refine_log(self, cap: int = 64) -> np.ndarray:
        """Rows: round, outer maxresid before it, Delta_P, Delta_D, inner
        iterations, inner status, inner maxresid, seconds since start, ended
        early for stalling (1/0), refined point accepted (1/0)."""
        buf = np.zeros((cap, 10))
        cnt = C.c_int(0)
        L.check(self.lib.pdhg_refine_log(self.ctx, buf.ctypes.data_as(C.c_void_p),
                                         cap, C.byref(cnt)), self.ctx)
        return buf[:min(cnt.value, cap)]

    # ------------------------------------------------------------- kernels
    def spmv(self, which: int, vec, scaled: bool = False, precision: int = L.FP64):
        nin = self.n if which == 0 else self.m
        nout = self.m if which == 0 else self.n
        a = _Arg(vec, np.float64, nin, "vec")
        out, po, mem = self._out(nout, a.mem == L.MEM_DEVICE)
        L.check(self.lib.pdhg_spmv(self.ctx, which, int(scaled), precision, a.ptr,
                                   po, mem), self.ctx)
        return out

    def spmv_noalloc(self, which: int, vec, scaled: bool = False,
                     precision: int = L.FP64, out=None):
        """pdhg_spmv_noalloc: the same product with the library's fixed
        device scratch as staging.  With a device `vec` and a device `out`
        (torch tensors on this GPU) nothing is allocated anywhere."""
        nin = self.n if which == 0 else self.m
        nout = self.m if which == 0 else self.n
        a = _Arg(vec, np.float64, nin, "vec")
        if out is None:
            out, po, mem = self._out(nout, a.mem == L.MEM_DEVICE)
        else:
            # written in place: must already be float64, contiguous, nout long
            if _is_torch(out):
                ok = (out.dtype == _torch().float64 and out.is_contiguous()
                      and out.numel() == nout)
                po = C.c_void_p(out.data_ptr())
                mem = L.MEM_DEVICE if out.is_cuda else L.MEM_HOST
            else:
                ok = (isinstance(out, np.ndarray) and out.dtype == np.float64
                      and out.flags.c_contiguous and out.flags.writeable
                      and out.size == nout)
                po, mem = (out.ctypes.data_as(C.c_void_p) if ok else None), L.MEM_HOST
            if not ok:
                raise ValueError(f"out: expected a contiguous float64 array of {nout}")
            if mem != a.mem:
                raise ValueError("vec and out must both be host or both device")
        L.check(self.lib.pdhg_spmv_noalloc(self.ctx, which, int(scaled), precision,
                                           a.ptr, po, mem), self.ctx)
        return out

    def gather_probe(self, table_entries: int, precision: int = L.FP64,
                     panels: int = 1, stream_nt: int = 0,
                     n_gathers: int = 1 << 25, reps: int = 5) -> float:
        """pdhg_gather_probe: random gathers per second from a table of
        table_entries values, each XCD confined to 1/panels of it."""
        r = C.c_double(0.0)
        L.check(self.lib.pdhg_gather_probe(self.ctx, int(table_entries), precision,
                                           panels, stream_nt, int(n_gathers), reps,
                                           C.byref(r)), self.ctx)
        return r.value

    def bin_stats(self, which: int):
        out = np.zeros(3, dtype=np.int64)
        L.check(self.lib.pdhg_bin_stats(self.ctx, which, out.ctypes.data_as(C.c_void_p)),
                self.ctx)
        return out

    def panel_count(self, which: int) -> int:
        out = C.c_int(0)
        L.check(self.lib.pdhg_panel_count(self.ctx, which, C.byref(out)), self.ctx)
        return out.value

    def profile(self, enable: bool = True):
        L.check(self.lib.pdhg_profile(self.ctx, int(enable)), self.ctx)

    def kernel_times(self, reset: bool = False) -> dict:
        buf = (L.KernelTime * 8)()
        cnt = C.c_int(0)
        L.check(self.lib.pdhg_kernel_times(self.ctx, buf, 8, C.byref(cnt), int(reset)),
                self.ctx)
        return {buf[i].name.decode(): dict(launches=buf[i].launches,
                                           total_ms=buf[i].total_ms)
                for i in range(cnt.value)}

    # ------------------------------------------------------------- adjoint
    def unrolled_forward(self, K: int, ckpt_every: int, tau: float, sigma: float,
                         precision: int = L.FP64, x0=None, y0=None,
                         device: bool = False):
        ax = _Arg(x0, np.float64, self.n, "x0")
        ay = _Arg(y0, np.float64, self.m, "y0")
        xK, pK, mem = self._out(self.n, device)
        if ax.ptr is not None and ax.mem != mem:
            raise ValueError("x0 and the output must live in the same memory")
        tape = C.c_void_p()
        L.check(self.lib.pdhg_unrolled_forward(self.ctx, K, ckpt_every, precision,
                                               tau, sigma, ax.ptr, ay.ptr, pK, mem,
                                               C.byref(tape)), self.ctx)
        t = Tape(self, tape)
        import weakref
        self._tapes = [r for r in self._tapes if r() is not None]
        self._tapes.append(weakref.ref(t))
        return xK, t


class Tape:
    def __init__(self, solver: Solver, handle):
        self.solver = solver
        self.h = handle

    def backward(self, gxK, device: bool = False):
        s = self.solver
        if s is None or not self.h or not s.ctx:
            raise L.PDHGError(-6, "tape was freed or its solver closed")
        a = _Arg(gxK, np.float64, s.n, "gxK")
        dev = a.mem == L.MEM_DEVICE
        gc, pc, mem = s._out(s.n, dev)
        gb, pb, _ = s._out(s.m, dev)
        gA, pA, _ = s._out(s.nnz, dev)
        L.check(s.lib.pdhg_unrolled_backward(self.h, a.ptr, pc, pb, pA, mem), s.ctx)
        return gc, gb, gA

    def free(self):
        if self.h:
            self.solver.lib.pdhg_tape_free(self.h)
            self.h = None
        self.solver = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
