"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid problems during host-side validation."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads
from paper_2407_14013_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in ("wcsdp.h", "wcsdp_linalg.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for mt in re.finditer(r"\b(sdp_\w+|wc_\w+)\s*\(", text):
            names.add(mt.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    declared = declared_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
    assert declared == set(L.exported_names())


def test_default_options():
    o = L.SdpOptions()
    L.lib().sdp_default_options(C.byref(o))
    assert o.rank_max == 10 and o.inner_tol == 1e-10 and o.gap_tol == 1e-8 and o.step_frac == 0.98
    assert o.solver == L.SDP_SOLVER_PCG and o.inner_prec == L.SDP_PREC_F64
    assert o.max_refine == 20 and o.refine_tol == 0.0 and o.lp_top_max == 2048


def _setup_status(problem, opts=None):
    lib = L.lib()
    keep = []

    def host(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(C.c_void_p)

    p = L.SdpProblem()
    p.n, p.m = problem["n"], problem["m"]
    p.a_kind = L.SDP_A_DENSE if problem["kind"] == "dense" else L.SDP_A_ENTRY
    p.b = host(problem["b"], np.float64)
    p.C = host(problem["C"], np.float64)
    if problem["kind"] == "dense":
        p.A = host(problem["A"], np.float64)
    else:
        p.jk = host(problem["jk"], np.int32)
    p.on_device = 0
    ctx = C.c_void_p()
    st = lib.sdp_setup(C.byref(p), C.byref(opts) if opts is not None else None, None, C.byref(ctx))
    return st, lib.sdp_last_error(None).decode(), ctx


@pytest.mark.parametrize(
    "mutate,needle",
    [
        (lambda p: p.update(n=1), "n must be"),
        (lambda p: p["b"].__setitem__(0, np.nan), "b has a non-finite"),
        (lambda p: p["C"].__setitem__((0, 1), 5.0), "C is not symmetric"),
        (lambda p: p["A"].__setitem__((0, 1), 3.0), "is not symmetric"),
        (lambda p: p["A"].__setitem__((2, 0), np.inf), "non-finite"),
    ],
)
def test_setup_rejects_invalid_dense(mutate, needle):
    p = workloads.gaussian_sensing(5, 1, 6, seed=0)
    p["C"] = p["C"].copy()
    mutate(p)
    st, msg, ctx = _setup_status(p)
    assert st == L.SDP_EINVAL and needle in msg and not ctx.value


@pytest.mark.parametrize(
    "mutate,needle",
    [
        (lambda p: p["jk"].__setitem__((0, 0), 7), "0 <= j <= k < n"),
        (lambda p: p["jk"].__setitem__(1, p["jk"][0]), "distinct"),
        (lambda p: p["jk"].__setitem__((0, 1), 99), "0 <= j <= k < n"),
    ],
)
def test_setup_rejects_invalid_entries(mutate, needle):
    p = workloads.matrix_completion(6, 1, 8, seed=1)
    p["jk"] = p["jk"].copy()
    if p["jk"][0, 0] == p["jk"][0, 1]:
        p["jk"][0] = [0, 5]
    mutate(p)
    st, msg, ctx = _setup_status(p)
    assert st == L.SDP_EINVAL and needle in msg


def test_setup_rejects_too_many_constraints():
    p = workloads.gaussian_sensing(3, 1, 6, seed=0)
    p["m"] = 7
    p["b"] = np.zeros(7)
    p["A"] = np.vstack([p["A"], p["A"][:1]])
    st, msg, _ = _setup_status(p)
    assert st == L.SDP_EINVAL and "n(n+1)/2" in msg


def test_setup_rejects_bad_options():
    lib = L.lib()
    o = L.SdpOptions()
    lib.sdp_default_options(C.byref(o))
    o.step_frac = 1.5
    p = L.SdpProblem()
    ctx = C.c_void_p()
    st = lib.sdp_setup(C.byref(p), C.byref(o), None, C.byref(ctx))
    assert st == L.SDP_EINVAL and "step_frac" in lib.sdp_last_error(None).decode()


@pytest.mark.parametrize(
    "field,value,needle",
    [
        ("inner_prec", 3, "inner_prec must be"),
        ("refine_tol", 1.5, "refine_tol must lie"),
        ("max_refine", -1, "max_refine must be"),
        ("step_frac", 1.0, "step_frac must lie"),
        ("solver", 7, "solver must be"),
    ],
)
def test_setup_rejects_invalid_options(field, value, needle):
    # option checks run before any device work, so they are testable without a GPU
    o = L.SdpOptions()
    L.lib().sdp_default_options(C.byref(o))
    setattr(o, field, value)
    st, msg, ctx = _setup_status(workloads.gaussian_sensing(5, 1, 6, seed=0), o)
    assert st == L.SDP_EINVAL and needle in msg and not ctx.value


def test_minres_requires_fp64_operator():
    o = L.SdpOptions()
    L.lib().sdp_default_options(C.byref(o))
    o.solver = L.SDP_SOLVER_MINRES
    o.inner_prec = L.SDP_PREC_F32
    st, msg, ctx = _setup_status(workloads.gaussian_sensing(5, 1, 6, seed=0), o)
    assert st == L.SDP_EINVAL and "MINRES runs with the FP64 operator" in msg and not ctx.value
