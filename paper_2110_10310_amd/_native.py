"""ctypes loader for liblbx.so (the C ABI declared in include/lbx.h).

The library is built in-tree by ``paper_2110_10310_amd.build``.  There is no
fallback: if the shared library is missing or does not load, importing this
module raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbx.so")

LB_OK = 0
LB_EINVAL = -1
LB_ENOMEM = -2
LB_EDEVICE = -3
LB_EUNSUPPORTED = -4
LB_ENONFINITE = -5

LB_J_FROB = 0
LB_J_TR = 1
LB_J_NM = 2

LB_OP_IMR_STEP = 0
LB_OP_FORWARD = 1
LB_OP_GRADIENT = 2
LB_OP_BACKWARD = 3

LB_OPT_PATH = 0
LB_OPT_SOLVE_TOL = 1
LB_OPT_PROFILE = 2
LB_OPT_TILE = 3
LB_OPT_TILE_KI = 4
LB_OPT_GRAPH = 5
LB_OPT_HISTORY = 6
LB_OPT_SYNC = 7
LB_OPT_SWEEPS = 8
LB_OPT_FUSE_GRAD = 9

LB_NOALLOC_SCRATCH_BYTES = 67108864
LB_NOALLOC_MAX_ENTRIES = 2064384
LB_NOALLOC_MAX_SYSTEMS = 256

LB_KERNEL_LDS_FORWARD = 0
LB_KERNEL_LDS_ADJOINT = 1
LB_KERNEL_SWEEP = 2
LB_KERNEL_STREAM_GRAD = 3
LB_KERNEL_COUNT = 4

# Every function the header declares, with its ctypes signature.
_i32 = C.c_int32
_p = C.c_void_p
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class SystemDesc(C.Structure):
    _fields_ = [
        ("Q", _i32), ("nlev", _ip), ("detuning", _dp), ("selfkerr", _dp),
        ("crosskerr", _dp), ("T1", _dp), ("T2", _dp), ("Ns", _i32), ("Nf", _i32),
        ("carrier", _dp), ("T", C.c_double), ("NT", _i32), ("jc", _dp), ("rotfreq", _dp),
    ]


SIGNATURES = {
    "lb_plan_create": (C.c_int, [C.POINTER(SystemDesc), _i32, C.POINTER(_p)]),
    "lb_plan_destroy": (None, [_p]),
    "lb_plan_info": (C.c_int, [_p, _i32, _ip, _ip, _ip]),
    "lb_plan_set_option": (C.c_int, [_p, _i32, C.c_double]),
    "lb_workspace_bytes": (C.c_int, [_p, _i32, _ip, _i32, C.POINTER(C.c_size_t)]),
    "control_table": (C.c_int, [_p, _i32, _p, _p, _p]),
    "lindblad_apply": (C.c_int, [_p, _i32, C.c_double, _p, _p, _p, _i32, _i32, _p]),
    "imr_step": (C.c_int, [_p, _i32, _i32, _p, _p, _p, _i32, _i32, _p, C.c_size_t, _p]),
    "forward_solve": (C.c_int, [_p, _p, _p, _p, _ip, _p, _i32, _p, C.c_size_t, _p]),
    "objective": (C.c_int, [_p, _i32, _p, _p, _p, _ip, C.c_double, _p, _p, _p, _p,
                            C.c_size_t, _p]),
    "adjoint_gradient": (C.c_int, [_p, _i32, _p, _p, _p, _p, _ip, C.c_double, C.c_double, C.c_double, _i32,
                                   _p, _p, _p, _p, C.c_size_t, _p]),
    "adjoint_backward": (C.c_int, [_p, _i32, _p, _p, _i32, _p, _p, _ip, C.c_double, _p, _p,
                                   _p, C.c_size_t, _p]),
    "lb_trajectory_bytes": (C.c_int, [_p, _ip, _i32, C.POINTER(C.c_size_t)]),
    "lb_status": (C.c_int, [_p, _p, _p]),
    "imr_step_noalloc": (C.c_int, [_p, _i32, _i32, _p, _p, _p, _i32, _i32, _p]),
    "lb_profile_read": (C.c_int, [_p, _i32, C.POINTER(C.c_int64), C.POINTER(C.c_double), _i32]),
    "lb_profile_work": (C.c_int, [_p, _i32, C.POINTER(C.c_int64)]),
    "sweep_counts": (C.c_int, [_p, _p, _ip, _p]),
    "lb_autotune": (C.c_int, [_p, _p, _ip, _p, C.c_size_t, _p, _ip]),
    "lb_last_error": (C.c_char_p, []),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2110_10310_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class LbxError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib.lb_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with code {code}: {msg}")
        self.code = code


def check(code: int, where: str) -> None:
    if code != LB_OK:
        raise LbxError(code, where)
