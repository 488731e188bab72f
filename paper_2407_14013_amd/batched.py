"""Python binding of sdp_solve_batched / sdp_autotune_batched (argument marshalling only)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .api import SdpError, _stream_ptr, default_options


def _problems(problems, keep):
    arr = (L.SdpProblem * len(problems))()
    for i, p in enumerate(problems):
        if p["kind"] != "dense":
            raise ValueError("the batched solver takes dense constraint matrices")
        A = np.ascontiguousarray(p["A"], dtype=np.float64)
        b = np.ascontiguousarray(p["b"], dtype=np.float64)
        Cm = np.ascontiguousarray(p["C"], dtype=np.float64)
        keep += [A, b, Cm]
        q = arr[i]
        q.n, q.m, q.a_kind, q.on_device = int(p["n"]), int(p["m"]), L.SDP_A_DENSE, 0
        q.A = A.ctypes.data_as(C.c_void_p)
        q.b = b.ctypes.data_as(C.c_void_p)
        q.C = Cm.ctypes.data_as(C.c_void_p)
    return arr


def autotune(problems, stream=None, **opts):
    """Per-instance configurations (rows_per_wave, aq_group, gemm_tile) and the buckets' winning times."""
    keep = []
    probs = _problems(problems, keep)
    o = default_options(**opts)
    tune = (L.SdpBatchTune * len(problems))()
    ms = (C.c_double * 3)()
    st = L.lib().sdp_autotune_batched(probs, len(problems), C.byref(o), _stream_ptr(stream), tune, ms)
    if st != L.SDP_OK:
        raise SdpError(st, L.lib().sdp_last_error(None).decode())
    return tune, list(ms)


def solve_batched(problems, tune=None, stream=None, want_y=False, **opts):
    """Solve every problem in one persistent launch; returns (results, [X_i], [y_i] or None)."""
    keep = []
    probs = _problems(problems, keep)
    o = default_options(**opts)
    dev = torch.device("cuda", torch.cuda.current_device())
    Xs = [torch.empty((int(p["n"]), int(p["n"])), dtype=torch.float64, device=dev) for p in problems]
    ys = [torch.empty(int(p["m"]), dtype=torch.float64, device=dev) for p in problems] if want_y else None
    xptr = (C.c_void_p * len(problems))(*[X.data_ptr() for X in Xs])
    yptr = (C.c_void_p * len(problems))(*[y.data_ptr() for y in ys]) if want_y else None
    res = (L.SdpResult * len(problems))()
    st = L.lib().sdp_solve_batched(probs, len(problems), C.byref(o), _stream_ptr(stream), res, xptr, yptr,
                                   tune if tune is not None else None)
    if st != L.SDP_OK:
        raise SdpError(st, L.lib().sdp_last_error(None).decode())
    # X_i is column-major n x n; symmetric, so the row-major view is the same matrix
    return [L.struct_dict(r) for r in res], Xs, ys
