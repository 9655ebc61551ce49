"""ctypes declarations of the libls C ABI (include/ls.h).

Argument marshalling only.  Loading fails loudly when libls.so has not been built: there is no
fallback implementation on this path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LS_LIBRARY", os.path.join(HERE, "libls.so"))

LS_C64 = 0
LS_C128 = 1
LS_SCRATCH_BYTES = 256 * 1024 * 1024   # fixed device scratch of ls_forward_farfield_noalloc
LS_OP_FORWARD, LS_OP_FARFIELD, LS_OP_GRAD, LS_OP_APPLY, LS_OP_PROX, LS_OP_INCIDENT = 0, 1, 2, 3, 4, 5

# every symbol declared in include/ls.h
EXPORTS = [
    "ls_strerror", "ls_last_error", "ls_kernel_bytes", "ls_init_workspace_bytes", "ls_green_init",
    "ls_ctx_destroy", "ls_workspace_bytes", "ls_apply_G", "ls_apply_A", "ls_forward", "ls_forward_farfield",
    "ls_forward_farfield_noalloc", "ls_farfield",
    "ls_farfield_adj", "ls_vjp", "ls_grad", "ls_batch_bytes", "ls_batch_create", "ls_batch_admit",
    "ls_batch_step", "ls_batch_poll", "ls_batch_release", "ls_batch_destroy", "ls_profile_pass",
    "ls_residual", "ls_grad_accumulate", "ls_prox_tv", "ls_fbs_extrapolate", "ls_tv_value",
    "ls_incident_field", "ls_forward_uin", "ls_detector_bytes", "ls_farfield_wide", "ls_farfield_wide_adj",
    "ls_pupil", "ls_decimate", "ls_vjp_rhs",
]


class Geom(C.Structure):
    _fields_ = [("n", C.c_int32), ("p", C.c_int32), ("kbh", C.c_double), ("xg", C.c_double),
                ("prec", C.c_int32), ("reserved", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("max_restarts", C.c_int32), ("x0_mode", C.c_int32),
                ("reserved", C.c_int32), ("breakdown", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("matvecs", C.c_int32), ("restarts", C.c_int32),
                ("relres_rec", C.c_double), ("relres_true", C.c_double), ("time_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


class LSError(RuntimeError):
    pass


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libls.so not found at {LIB_PATH}: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'` (no fallback exists)")
    lib = C.CDLL(LIB_PATH)
    vp, sz, i32, dp = C.c_void_p, C.c_size_t, C.c_int32, C.POINTER(C.c_double)
    P = C.POINTER
    sig = {
        "ls_strerror": (C.c_char_p, [C.c_int]),
        "ls_last_error": (C.c_char_p, []),
        "ls_kernel_bytes": (C.c_int, [P(Geom), P(sz)]),
        "ls_init_workspace_bytes": (C.c_int, [P(Geom), P(sz)]),
        "ls_green_init": (C.c_int, [P(Geom), vp, sz, vp, sz, vp, P(vp)]),
        "ls_ctx_destroy": (None, [vp]),
        "ls_workspace_bytes": (C.c_int, [vp, i32, i32, P(sz)]),
        "ls_apply_G": (C.c_int, [vp, vp, vp, i32, vp, sz, vp]),
        "ls_apply_A": (C.c_int, [vp, vp, vp, vp, i32, vp, sz, vp]),
        "ls_forward": (C.c_int, [vp, vp, i32, dp, vp, P(SolveOpts), P(SolveInfo), vp, sz, vp]),
        "ls_forward_farfield": (C.c_int, [vp, vp, i32, dp, vp, vp, P(SolveOpts), P(SolveInfo), vp, sz, vp]),
        "ls_forward_farfield_noalloc": (C.c_int, [vp, vp, i32, dp, vp, vp, P(SolveOpts), P(SolveInfo), vp]),
        "ls_farfield": (C.c_int, [vp, vp, vp, i32, vp, vp, sz, vp]),
        "ls_farfield_adj": (C.c_int, [vp, vp, i32, i32, vp, vp, sz, vp]),
        "ls_vjp": (C.c_int, [vp, vp, vp, i32, vp, vp, P(SolveOpts), P(SolveInfo), vp, sz, vp]),
        "ls_grad": (C.c_int, [vp, vp, i32, dp, vp, vp, dp, P(SolveOpts), P(SolveInfo), vp, sz, vp]),
        "ls_batch_bytes": (C.c_int, [vp, i32, P(sz)]),
        "ls_batch_create": (C.c_int, [vp, i32, vp, sz, P(SolveOpts), P(vp)]),
        "ls_batch_admit": (C.c_int, [vp, i32, vp, dp, vp, vp, vp]),
        "ls_batch_step": (C.c_int, [vp, i32, vp]),
        "ls_batch_poll": (C.c_int, [vp, P(i32), P(SolveInfo)]),
        "ls_batch_release": (C.c_int, [vp, i32]),
        "ls_batch_destroy": (None, [vp]),
        "ls_profile_pass": (C.c_int, [vp, vp, vp, i32, i32, i32, vp, sz, vp]),
        "ls_residual": (C.c_int, [vp, vp, vp, i32, i32, vp, vp, vp, vp]),
        "ls_grad_accumulate": (C.c_int, [vp, vp, vp, i32, vp, vp, i32, vp]),
        "ls_prox_tv": (C.c_int, [vp, vp, vp, C.c_double, C.c_double, i32, i32, vp, vp, sz, vp]),
        "ls_fbs_extrapolate": (C.c_int, [vp, vp, vp, C.c_double, vp, vp]),
        "ls_tv_value": (C.c_int, [vp, vp, dp, vp, sz, vp]),
        "ls_incident_field": (C.c_int, [vp, vp, dp, i32, i32, vp, vp, sz, vp]),
        "ls_forward_uin": (C.c_int, [vp, vp, i32, vp, vp, P(SolveOpts), P(SolveInfo), vp, sz, vp]),
        "ls_detector_bytes": (C.c_int, [vp, i32, P(sz)]),
        "ls_farfield_wide": (C.c_int, [vp, i32, vp, vp, i32, vp, vp, sz, vp]),
        "ls_farfield_wide_adj": (C.c_int, [vp, i32, vp, i32, i32, vp, vp, sz, vp]),
        "ls_pupil": (C.c_int, [vp, i32, vp, i32, C.c_double, C.c_double, i32, vp, vp, sz, vp]),
        "ls_decimate": (C.c_int, [vp, i32, i32, vp, i32, vp, i32, vp]),
        "ls_vjp_rhs": (C.c_int, [vp, vp, vp, i32, vp, vp, P(SolveOpts), P(SolveInfo), vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, what: str) -> None:
    if rc != 0:
        lib = load()
        raise LSError(f"{what}: {lib.ls_strerror(rc).decode()} ({rc}) {lib.ls_last_error().decode()}")
