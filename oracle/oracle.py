"""ctypes front end of the FP64 CPU oracle (``pdhg_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg load this module; the product path never
does.  It imports nothing from the HIP package and marshals numpy arrays only.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdhg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-ffp-contract=off",
          "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(LIB) or \
            os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("ruiz_passes", C.c_int32), ("power_iters", C.c_int32),
                ("eval_every", C.c_int32), ("literal_snapshots", C.c_int32),
                ("variant", C.c_int32), ("pad0_", C.c_int32),
                ("eps_rel", C.c_double), ("eta", C.c_double),
                ("omega0", C.c_double), ("eta_factor", C.c_double),
                ("beta_suff", C.c_double), ("beta_nec", C.c_double),
                ("beta_art", C.c_double), ("omega_theta", C.c_double),
                ("reflect", C.c_double),
                ("max_iters", C.c_int64), ("time_limit_s", C.c_double),
                ("n_levels", C.c_int32), ("pad_", C.c_int32),
                ("levels", C.POINTER(C.c_double)),
                ("omega_rule", C.c_int32), ("pad2_", C.c_int32),
                ("pid_kp", C.c_double), ("pid_ki", C.c_double),
                ("pid_kd", C.c_double), ("stop_on", C.c_int32),
                ("polish", C.c_int32), ("polish_frac", C.c_double)]


class KKT(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("rel_p", "rel_d", "rel_gap", "maxresid", "pobj", "dobj",
                 "norm_rp", "norm_rd", "rp_inf", "rd_inf")]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("candidate", C.c_int32),
                ("iters", C.c_int64), ("restarts", C.c_int32),
                ("n_snap", C.c_int32), ("n_log", C.c_int32),
                ("polish_attempts", C.c_int32), ("sigma_hat", C.c_double),
                ("eta", C.c_double), ("omega0", C.c_double),
                ("omega", C.c_double), ("tau", C.c_double),
                ("sigma", C.c_double), ("t_setup", C.c_double),
                ("t_iter", C.c_double), ("kkt", KKT),
                ("polish_iters", C.c_int64)]


class Snap(C.Structure):
    _fields_ = [("level", C.c_double), ("iter", C.c_int64),
                ("maxresid", C.c_double), ("candidate", C.c_int32),
                ("pad_", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or \
                os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = C.CDLL(LIB)
        _lib.or_power.restype = C.c_double
    return _lib


def _p(a: Optional[np.ndarray], dt=np.float64):
    if a is None:
        return None
    assert a.dtype == dt and a.flags.c_contiguous, (a.dtype, dt)
    return a.ctypes.data_as(C.c_void_p)


def _csr(lp):
    rp = np.ascontiguousarray(lp.a_rp, dtype=np.int64)
    ci = np.ascontiguousarray(lp.a_ci, dtype=np.int32)
    v = np.ascontiguousarray(lp.a_v, dtype=np.float64)
    return rp, ci, v


DEFAULTS = dict(ruiz_passes=10, power_iters=100, eval_every=64,
                literal_snapshots=0, variant=0, eps_rel=1e-6, eta=0.0,
                omega0=0.0, eta_factor=0.9, beta_suff=0.2, beta_nec=0.8,
                beta_art=0.36, omega_theta=0.5, reflect=1.0, max_iters=10**9,
                time_limit_s=3600.0, omega_rule=0, pid_kp=0.99, pid_ki=0.01,
                pid_kd=0.0, stop_on=0, polish=0, polish_frac=0.125)


def make_params(levels: Sequence[float] = (), **kw) -> tuple:
    d = dict(DEFAULTS)
    d.update(kw)
    lv = np.ascontiguousarray(np.asarray(levels, dtype=np.float64))
    p = Params(**{k: d[k] for k in DEFAULTS}, pad0_=0, n_levels=len(lv), pad_=0, pad2_=0,
               levels=lv.ctypes.data_as(C.POINTER(C.c_double)))
    return p, lv


def ruiz(lp, passes: int = 10):
    rp, ci, v = _csr(lp)
    dr = np.empty(lp.m)
    dc = np.empty(lp.n)
    vs = np.empty(lp.nnz)
    rc = lib().or_ruiz(C.c_int64(lp.m), C.c_int64(lp.n), _p(rp, np.int64),
                       _p(ci, np.int32), _p(v), C.c_int32(passes), _p(dr),
                       _p(dc), _p(vs))
    assert rc == 0
    return dr, dc, vs


def power(lp, vals: np.ndarray, iters: int = 100) -> float:
    rp, ci, _ = _csr(lp)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    return lib().or_power(C.c_int64(lp.m), C.c_int64(lp.n), _p(rp, np.int64),
                          _p(ci, np.int32), _p(vals), C.c_int32(iters))


def kkt(lp, x, y, l=None, want_z=False):
    rp, ci, v = _csr(lp)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.empty(lp.n) if want_z else None
    out = KKT()
    rc = lib().or_kkt(C.c_int64(lp.m), C.c_int64(lp.n), _p(rp, np.int64),
                      _p(ci, np.int32), _p(v), _p(np.ascontiguousarray(lp.b)),
                      _p(np.ascontiguousarray(lp.c)),
                      _p(None if l is None else np.ascontiguousarray(l, dtype=np.float64)),
                      _p(x), _p(y), _p(z), C.byref(out))
    assert rc == 0
    d = out.asdict()
    if want_z:
        d["z"] = z
    return d


def alg1_levels(eps_cross: float, eps_rel: float, cap: int = 64):
    out = np.zeros(cap)
    k = lib().or_alg1_levels(C.c_double(eps_cross), C.c_double(eps_rel),
                             _p(out), C.c_int(cap))
    return out[:k].tolist()


@dataclass
class SolveResult:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    info: dict
    kkt: dict
    snaps: list
    snap_x: Optional[np.ndarray]
    snap_y: Optional[np.ndarray]
    snap_z: Optional[np.ndarray]
    trace_x: Optional[np.ndarray]
    trace_y: Optional[np.ndarray]
    eval_log: np.ndarray


def solve(lp, levels: Sequence[float] = (), l=None, x0=None, y0=None,
          trace_k: int = 0, keep_snap_vectors: bool = False,
          log_cap: int = 4096, b=None, c=None, **kw) -> SolveResult:
    """Run the oracle PDHG.  Keyword arguments override DEFAULTS."""
    rp, ci, v = _csr(lp)
    m, n = lp.m, lp.n
    bb = np.ascontiguousarray(lp.b if b is None else b, dtype=np.float64)
    cc = np.ascontiguousarray(lp.c if c is None else c, dtype=np.float64)
    prm, lv = make_params(levels, **kw)
    info = Info()
    x = np.empty(n); y = np.empty(m); z = np.empty(n)
    nl = max(len(lv), 1)
    snaps = (Snap * nl)()
    sx = np.empty(nl * n) if keep_snap_vectors else None
    sy = np.empty(nl * m) if keep_snap_vectors else None
    sz = np.empty(nl * n) if keep_snap_vectors else None
    tx = np.empty(max(trace_k, 1) * n) if trace_k else None
    ty = np.empty(max(trace_k, 1) * m) if trace_k else None
    elog = np.zeros(log_cap * 8)
    cvt = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    rc = lib().or_solve(C.c_int64(m), C.c_int64(n), _p(rp, np.int64),
                        _p(ci, np.int32), _p(v), _p(bb), _p(cc), _p(cvt(l)),
                        _p(cvt(x0)), _p(cvt(y0)), C.byref(prm), C.byref(info),
                        _p(x), _p(y), _p(z), snaps, _p(sx), _p(sy), _p(sz),
                        C.c_int32(trace_k), _p(tx), _p(ty), C.c_int32(log_cap),
                        _p(elog))
    if rc != 0:
        raise ValueError(f"oracle or_solve failed: {rc}")
    idict = {k: getattr(info, k) for k, _ in Info._fields_ if k != "kkt"}
    ns = info.n_snap
    slist = [dict(level=snaps[i].level, iter=snaps[i].iter,
                  maxresid=snaps[i].maxresid, candidate=snaps[i].candidate)
             for i in range(ns)]
    nlog = min(info.n_log, log_cap)
    return SolveResult(
        x, y, z, idict, info.kkt.asdict(), slist,
        None if sx is None else sx.reshape(nl, n)[:ns],
        None if sy is None else sy.reshape(nl, m)[:ns],
        None if sz is None else sz.reshape(nl, n)[:ns],
        None if tx is None else tx.reshape(trace_k, n),
        None if ty is None else ty.reshape(trace_k, m),
        elog.reshape(-1, 8)[:nlog])


def refine(lp, outer_eps: float = 1e-8, max_rounds: int = 8,
           cap_log2: int = 10, progress: float = 1e-2, **inner_kw):
    """FP64 iterative refinement with FP64 inner solves (logic check)."""
    rp, ci, v = _csr(lp)
    kw = dict(eps_rel=1e-4)
    kw.update(inner_kw)
    prm, lv = make_params((), **kw)
    x = np.empty(lp.n); y = np.empty(lp.m)
    K = KKT()
    rounds = C.c_int32(0)
    inner = C.c_int64(0)
    rlog = np.zeros(4 * (max_rounds + 1))
    st = lib().or_refine(C.c_int64(lp.m), C.c_int64(lp.n), _p(rp, np.int64),
                         _p(ci, np.int32), _p(v),
                         _p(np.ascontiguousarray(lp.b)),
                         _p(np.ascontiguousarray(lp.c)), C.byref(prm),
                         C.c_double(outer_eps), C.c_double(progress),
                         C.c_int32(max_rounds),
                         C.c_int32(cap_log2), _p(x), _p(y), C.byref(K),
                         C.byref(rounds), C.byref(inner), _p(rlog))
    return dict(status=st, x=x, y=y, kkt=K.asdict(), rounds=rounds.value,
                inner_iters=inner.value,
                round_log=rlog.reshape(-1, 4)[:rounds.value + 1])


def unrolled(lp, dr, dc, tau, sigma, K, xt, x0=None, y0=None, vals=None,
             b=None, c=None):
    """K plain steps + reverse pass: returns (xK, loss, gc, gb, gA)."""
    rp, ci, v = _csr(lp)
    if vals is not None:
        v = np.ascontiguousarray(vals, dtype=np.float64)
    bb = np.ascontiguousarray(lp.b if b is None else b, dtype=np.float64)
    cc = np.ascontiguousarray(lp.c if c is None else c, dtype=np.float64)
    xK = np.empty(lp.n); gc = np.empty(lp.n); gb = np.empty(lp.m)
    gA = np.empty(lp.nnz)
    loss = C.c_double(0.0)
    cvt = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    rc = lib().or_unrolled(C.c_int64(lp.m), C.c_int64(lp.n), _p(rp, np.int64),
                           _p(ci, np.int32), _p(v), _p(bb), _p(cc),
                           _p(cvt(dr)), _p(cvt(dc)), C.c_double(tau),
                           C.c_double(sigma), C.c_int32(K), _p(cvt(x0)),
                           _p(cvt(y0)), _p(cvt(xt)), _p(xK), C.byref(loss),
                           _p(gc), _p(gb), _p(gA))
    assert rc == 0
    return xK, loss.value, gc, gb, gA


def unrolled_fwd(lp, dr, dc, tau, sigma, K, vals=None, b=None, c=None):
    """Forward only: returns (xK, mask_hash)."""
    rp, ci, v = _csr(lp)
    if vals is not None:
        v = np.ascontiguousarray(vals, dtype=np.float64)
    bb = np.ascontiguousarray(lp.b if b is None else b, dtype=np.float64)
    cc = np.ascontiguousarray(lp.c if c is None else c, dtype=np.float64)
    xK = np.empty(lp.n)
    h = C.c_uint64(0)
    cvt = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    rc = lib().or_unrolled_fwd(C.c_int64(lp.m), C.c_int64(lp.n),
                               _p(rp, np.int64), _p(ci, np.int32), _p(v),
                               _p(bb), _p(cc), _p(cvt(dr)), _p(cvt(dc)),
                               C.c_double(tau), C.c_double(sigma),
                               C.c_int32(K), _p(xK), C.byref(h))
    assert rc == 0
    return xK, h.value
