"""The C-ABI library loads without a GPU, exports every symbol that
include/lbx.h declares, and rejects invalid arguments before any device
call.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["lindblad_apply", "imr_step", "forward_solve", "objective", "adjoint_gradient",
              "control_table", "lb_plan_create", "lb_plan_destroy", "lb_workspace_bytes",
              "lb_last_error", "lb_plan_info", "lb_plan_set_option"]:
        assert n in names


def test_library_exports_every_declared_symbol(built_lib):
    lib = C.CDLL(built_lib)
    for n in declared_functions():
        assert hasattr(lib, n), n
    from paper_2110_10310_amd import _native
    assert set(_native.SIGNATURES) == set(declared_functions())


def test_invalid_arguments_rejected_before_device_calls(built_lib):
    from paper_2110_10310_amd import _native as nat
    lib = nat.lib
    h = C.c_void_p()
    assert lib.lb_plan_create(None, 1, C.byref(h)) == nat.LB_EINVAL
    assert b"no systems" in lib.lb_last_error()
    d = (nat.SystemDesc * 1)()
    d[0].Q = 0
    assert lib.lb_plan_create(d, 1, C.byref(h)) == nat.LB_EINVAL
    assert b"Q must be" in lib.lb_last_error()
    d[0].Q = 13
    assert lib.lb_plan_create(d, 1, C.byref(h)) == nat.LB_EINVAL
    size = C.c_size_t()
    b = (C.c_int32 * 1)(1)
    assert lib.lb_workspace_bytes(None, 0, b, 1, C.byref(size)) == nat.LB_EINVAL
    assert lib.lindblad_apply(None, 0, 0.0, None, None, None, 1, 0, None) == nat.LB_EINVAL
    assert lib.adjoint_gradient(None, 0, None, None, None, None, None, 0.0, 0.0, 1.0, 1, None, None, None,
                                None, 0, None) == nat.LB_EINVAL
    assert lib.lb_plan_set_option(None, 0, 0.0) == nat.LB_EINVAL
    assert lib.imr_step_noalloc(None, 0, 0, None, None, None, 1, 0, None) == nat.LB_EINVAL


def test_plan_validation_of_parameters(built_lib):
    import numpy as np
    from paper_2110_10310_amd import _native as nat
    lib = nat.lib

    def desc(**kw):
        Q = kw.get("Q", 1)
        arrs = dict(nlev=np.array(kw.get("nlev", [3] * Q), np.int32), det=np.zeros(Q), sk=np.zeros(Q),
                    ck=np.zeros(Q * Q), T1=np.full(Q, np.inf), T2=np.full(Q, np.inf),
                    car=np.zeros(Q))
        d = (nat.SystemDesc * 1)()
        d[0].Q = Q
        d[0].nlev = arrs["nlev"].ctypes.data_as(nat._ip)
        for f, k in (("detuning", "det"), ("selfkerr", "sk"), ("crosskerr", "ck"), ("T1", "T1"),
                     ("T2", "T2"), ("carrier", "car")):
            setattr(d[0], f, arrs[k].ctypes.data_as(nat._dp))
        d[0].Ns = kw.get("Ns", 5)
        d[0].Nf = 1
        d[0].T = kw.get("T", 1.0)
        d[0].NT = kw.get("NT", 10)
        return d, arrs

    h = C.c_void_p()
    for bad, msg in [(dict(Ns=2), b"Ns"), (dict(T=0.0), b"T must"), (dict(NT=0), b"NT"),
                     (dict(nlev=[40]), b"nlev"), (dict(T=float("nan")), b"T must")]:
        d, keep = desc(**bad)
        assert lib.lb_plan_create(d, 1, C.byref(h)) == nat.LB_EINVAL
        assert msg in lib.lb_last_error()
