"""ctypes binding of libpdhg.so (the C ABI in include/pdhg.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built; there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PDHG_LIB") or os.path.join(HERE, "libpdhg.so")

PDHG_OK = 0
ERRORS = {-1: "PDHG_E_ARG", -2: "PDHG_E_CSR", -3: "PDHG_E_TRANSPOSE",
          -4: "PDHG_E_DEVICE", -5: "PDHG_E_OOM", -6: "PDHG_E_STATE"}
STATUS = {0: "RUNNING", 1: "CONVERGED", 2: "ITER_LIMIT", 3: "TIME_LIMIT",
          4: "CANCELLED", 5: "NUMERICAL"}
MEM_HOST, MEM_DEVICE = 0, 1
FP64, FP32 = 0, 1
# device scratch of pdhg_spmv_noalloc (PDHG_SPMV_NOALLOC_MAX_BYTES)
SPMV_NOALLOC_MAX_BYTES = 64 << 20


class PDHGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("ruiz_passes", C.c_int32),
                ("power_iters", C.c_int32), ("eval_every", C.c_int32),
                ("literal_snapshots", C.c_int32), ("n_levels", C.c_int32),
                ("levels", C.POINTER(C.c_double)), ("eps_rel", C.c_double),
                ("eta", C.c_double), ("omega0", C.c_double),
                ("eta_factor", C.c_double), ("beta_suff", C.c_double),
                ("beta_nec", C.c_double), ("beta_art", C.c_double),
                ("omega_theta", C.c_double), ("max_iters", C.c_int64),
                ("time_limit_s", C.c_double), ("use_graph", C.c_int32),
                ("variant", C.c_int32), ("reflect", C.c_double),
                ("omega_rule", C.c_int32), ("pad_", C.c_int32),
                ("pid_kp", C.c_double), ("pid_ki", C.c_double),
                ("pid_kd", C.c_double), ("stop_on", C.c_int32),
                ("polish", C.c_int32), ("polish_frac", C.c_double)]


class KKT(C.Structure):
    _fields_ = [("rel_p", C.c_double), ("rel_d", C.c_double),
                ("rel_gap", C.c_double), ("maxresid", C.c_double),
                ("pobj", C.c_double), ("dobj", C.c_double),
                ("norm_rp", C.c_double), ("norm_rd", C.c_double),
                ("rp_inf", C.c_double), ("rd_inf", C.c_double),
                ("iter", C.c_int64), ("candidate", C.c_int32),
                ("pad_", C.c_int32)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("candidate", C.c_int32),
                ("iters", C.c_int64), ("restarts", C.c_int32),
                ("n_snap", C.c_int32), ("sigma_hat", C.c_double),
                ("eta", C.c_double), ("omega0", C.c_double),
                ("omega", C.c_double), ("tau", C.c_double),
                ("sigma", C.c_double), ("t_setup", C.c_double),
                ("t_iter", C.c_double), ("kkt", KKT),
                ("polish_attempts", C.c_int32), ("pad_", C.c_int32),
                ("polish_iters", C.c_int64)]

    def asdict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "kkt"}
        d["kkt"] = self.kkt.asdict()
        return d


class SnapInfo(C.Structure):
    _fields_ = [("level", C.c_double), ("iter", C.c_int64),
                ("maxresid", C.c_double), ("candidate", C.c_int32),
                ("pad_", C.c_int32), ("t_wall", C.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class RefineParams(C.Structure):
    _fields_ = [("outer_eps", C.c_double), ("inner_eps", C.c_double),
                ("max_rounds", C.c_int32), ("cap_log2", C.c_int32),
                ("max_inner_iters", C.c_int64), ("progress", C.c_double),
                ("inner_precision", C.c_int32), ("omega_carry", C.c_int32),
                ("stall_iters", C.c_int64)]


class RefineInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("rounds", C.c_int32),
                ("inner_iters", C.c_int64), ("t_total", C.c_double),
                ("kkt", KKT)]

    def asdict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "kkt"}
        d["kkt"] = self.kkt.asdict()
        return d


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64),
                ("total_ms", C.c_double)]


SNAP_CB = C.CFUNCTYPE(None, C.c_void_p, C.c_int, C.POINTER(SnapInfo),
                      C.POINTER(C.c_double), C.POINTER(C.c_double),
                      C.POINTER(C.c_double))
CROSSOVER_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.POINTER(SnapInfo),
                           C.POINTER(C.c_double), C.POINTER(C.c_double),
                           C.POINTER(C.c_double), C.POINTER(C.c_int32))

vp = C.c_void_p
i64 = C.c_int64
i32 = C.c_int
dbl = C.c_double

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "pdhg_params_default": (i32, [C.POINTER(Params)]),
    "pdhg_refine_params_default": (i32, [C.POINTER(RefineParams)]),
    "pdhg_alg1_levels": (i32, [dbl, dbl, vp, i32]),
    "pdhg_validate_csr": (i32, [i64, i64, i64, vp, vp, C.c_char_p, i32]),
    "pdhg_check_transpose": (i32, [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp,
                                   C.c_char_p, i32]),
    "pdhg_plan_bins": (i32, [i64, vp, i32, i64, i64, vp, i64]),
    "pdhg_create": (i32, [i32, vp, C.POINTER(vp)]),
    "pdhg_destroy": (None, [vp]),
    "pdhg_last_error": (C.c_char_p, [vp]),
    "pdhg_load": (i32, [vp, i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                        i32]),
    "pdhg_set_values": (i32, [vp, vp, i32]),
    "pdhg_set_rhs_obj": (i32, [vp, vp, vp, i32]),
    "pdhg_configure": (i32, [vp, C.POINTER(Params)]),
    "pdhg_set_iterate": (i32, [vp, vp, vp, i32]),
    "pdhg_iterate": (i32, [vp, i64, C.POINTER(i32)]),
    "pdhg_cancel": (i32, [vp]),
    "pdhg_get_info": (i32, [vp, C.POINTER(Info)]),
    "pdhg_residuals": (i32, [vp, i32, C.POINTER(KKT)]),
    "pdhg_get_iterate": (i32, [vp, vp, vp, vp, i32]),
    "pdhg_get_scaling": (i32, [vp, vp, vp, i32]),
    "pdhg_eval_log": (i32, [vp, vp, i32, C.POINTER(i32)]),
    "pdhg_snapshot_count": (i32, [vp, C.POINTER(i32)]),
    "pdhg_snapshot": (i32, [vp, i32, C.POINTER(SnapInfo), vp, vp, vp, i32]),
    "pdhg_set_snapshot_callback": (i32, [vp, SNAP_CB, vp]),
    "pdhg_concurrent_crossover": (i32, [vp, CROSSOVER_FN, vp, i32, i64,
                                        C.POINTER(i32), C.POINTER(i32)]),
    "pdhg_concurrent_crossover_refined": (i32, [vp, CROSSOVER_FN, vp, i32, vp, vp, vp, vp]),
    "pdhg_solve_refined": (i32, [vp, C.POINTER(RefineParams),
                                 C.POINTER(RefineInfo)]),
    "pdhg_refine_log": (i32, [vp, vp, i32, C.POINTER(i32)]),
    "pdhg_unrolled_forward": (i32, [vp, i32, i32, i32, dbl, dbl, vp, vp, vp,
                                    i32, C.POINTER(vp)]),
    "pdhg_unrolled_backward": (i32, [vp, vp, vp, vp, vp, i32]),
    "pdhg_tape_free": (None, [vp]),
    "pdhg_spmv": (i32, [vp, i32, i32, i32, vp, vp, i32]),
    "pdhg_spmv_noalloc": (i32, [vp, i32, i32, i32, vp, vp, i32]),
    "pdhg_gather_probe": (i32, [vp, i64, i32, i32, i32, i64, i32,
                                C.POINTER(C.c_double)]),
    "pdhg_set_tuning": (i32, [vp, C.c_char_p, i64]),
    "pdhg_bin_stats": (i32, [vp, i32, vp]),
    "pdhg_panel_count": (i32, [vp, i32, vp]),
    "pdhg_choose_panels": (i32, [i64, i64, i64]),
    "pdhg_cpu_steps": (i32, [i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, C.c_double,
                             C.c_double, i32, i32, vp, vp, vp]),
    "pdhg_plan_panels": (i32, [i64, i64, vp, vp, i32, vp, i32, vp, vp, vp, i64]),
    "pdhg_cpu_create": (i32, [i32, C.POINTER(vp)]),
    "pdhg_cpu_destroy": (None, [vp]),
    "pdhg_cpu_last_error": (C.c_char_p, [vp]),
    "pdhg_cpu_set_threads": (i32, [vp, i32]),
    "pdhg_cpu_load": (i32, [vp, i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    "pdhg_cpu_configure": (i32, [vp, C.POINTER(Params)]),
    "pdhg_cpu_iterate": (i32, [vp, i64, C.POINTER(i32)]),
    "pdhg_cpu_cancel": (i32, [vp]),
    "pdhg_cpu_get_info": (i32, [vp, C.POINTER(Info)]),
    "pdhg_cpu_get_iterate": (i32, [vp, vp, vp, vp]),
    "pdhg_cpu_get_scaling": (i32, [vp, vp, vp]),
    "pdhg_cpu_eval_log": (i32, [vp, vp, i32, C.POINTER(i32)]),
    "pdhg_cpu_snapshot_count": (i32, [vp, C.POINTER(i32)]),
    "pdhg_cpu_snapshot": (i32, [vp, i32, C.POINTER(SnapInfo), vp, vp, vp]),
    "pdhg_cpu_stream_bw": (i32, [i32, i64, i32, C.POINTER(C.c_double)]),
    "pdhg_profile": (i32, [vp, i32]),
    "pdhg_kernel_times": (i32, [vp, C.POINTER(KernelTime), i32,
                                C.POINTER(i32), i32]),
}

_lib = None


def lib():
    """Load libpdhg.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname as the
        # system one this library links; loading torch first makes the
        # library bind to that runtime, so torch's tensors and streams and
        # the library share one (loaded the other way round, the system
        # runtime has been seen to find no device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int, ctx=None):
    """Raise PDHGError for a negative return code, with the context's
    message when there is a context."""
    if rc < 0:
        msg = ""
        if ctx:
            m = lib().pdhg_last_error(ctx)
            msg = m.decode() if m else ""
        raise PDHGError(rc, msg)
    return rc


def check_create(rc: int):
    """check() for pdhg_create: the message of this thread's failed create."""
    if rc < 0:
        m = lib().pdhg_last_error(None)
        raise PDHGError(rc, m.decode() if m else "")
    return rc


def default_params(**kw) -> tuple:
    """Params struct with defaults overridden by kw; returns (params, keep)."""
    p = Params()
    check(lib().pdhg_params_default(C.byref(p)))
    keep = None
    levels = kw.pop("levels", None)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    if levels is not None and len(levels):
        keep = (C.c_double * len(levels))(*[float(t) for t in levels])
        p.levels = C.cast(keep, C.POINTER(C.c_double))
        p.n_levels = len(levels)
    return p, keep


def alg1_levels(eps_cross: float, eps_rel: float, cap: int = 64):
    buf = (C.c_double * cap)()
    k = check(lib().pdhg_alg1_levels(eps_cross, eps_rel,
                                     C.cast(buf, C.c_void_p), cap))
    return [buf[i] for i in range(k)]
