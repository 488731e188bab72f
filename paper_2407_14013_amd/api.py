"""Python binding of the C ABI: argument marshalling only.

Every computation happens in libwcsdp.so.  Device arrays are torch CUDA
float64 tensors; the C library sees their raw pointers and the current torch
stream.  Column-major n x n matrices from the library are returned as torch
tensors in the usual (row, column) orientation.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


class SdpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _stream_ptr(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t: torch.Tensor, name: str, numel: int | None = None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def default_options(**kw) -> L.SdpOptions:
    o = L.SdpOptions()
    L.lib().sdp_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Context:
    """One SDP instance on the GPU (wraps sdp_ctx)."""

    def __init__(self, problem: dict, options: L.SdpOptions | None = None, stream=None, **opt_kw):
        lib = L.lib()
        self._lib = lib
        self.n = int(problem["n"])
        self.m = int(problem["m"])
        self.kind = problem["kind"]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if options is None:
            options = default_options(**opt_kw)
        self.options = options
        keep = []
        p = L.SdpProblem()
        p.n, p.m = self.n, self.m
        p.a_kind = {"dense": L.SDP_A_DENSE, "entry": L.SDP_A_ENTRY, "sparse": L.SDP_A_SPARSE}[self.kind]

        def host(arr, dtype):
            a = np.ascontiguousarray(arr, dtype=dtype)
            keep.append(a)
            return a.ctypes.data_as(C.c_void_p)

        on_device = isinstance(problem["b"], torch.Tensor)
        p.on_device = 1 if on_device else 0
        spr = None
        if self.kind == "sparse":
            # entries on and above the diagonal per constraint (host arrays)
            sp = problem["sp"]
            spr = L.SdpSparseRows()
            spr.ptr = host(sp["ptr"], np.int32)
            spr.row = host(sp["row"], np.int32)
            spr.col = host(sp["col"], np.int32)
            spr.val = host(sp["val"], np.float64)
            spr.on_device = 0
            p.b = host(problem["b"].cpu().numpy() if on_device else problem["b"], np.float64)
            p.C = host(problem["C"].cpu().numpy() if on_device else problem["C"], np.float64)
            p.on_device = 0
        elif on_device:
            for key in ("b", "C") + (("A",) if self.kind == "dense" else ("jk",)):
                t = problem[key]
                if not t.is_contiguous() or not t.is_cuda:
                    raise ValueError(f"problem[{key!r}] must be a contiguous CUDA tensor")
                keep.append(t)
            p.b = C.c_void_p(problem["b"].data_ptr())
            p.C = C.c_void_p(problem["C"].data_ptr())
            if self.kind == "dense":
                p.A = C.c_void_p(problem["A"].data_ptr())
            else:
                p.jk = C.c_void_p(problem["jk"].data_ptr())
        else:
            p.b = host(problem["b"], np.float64)
            # C is symmetric, so row- and column-major layouts coincide
            p.C = host(problem["C"], np.float64)
            if self.kind == "dense":
                p.A = host(problem["A"], np.float64)
            else:
                p.jk = host(problem["jk"], np.int32)
        # nonnegative-orthant block (problem["lp"]: B by columns and the cost c)
        lpb = None
        self.ell = 0
        if problem.get("lp") is not None:
            lp = problem["lp"]
            self.ell = int(len(lp["c"]))
            lpb = L.SdpLpBlock()
            lpb.l = self.ell
            lpb.on_device = 0
            lpb.col_ptr = host(lp["ptr"], np.int32)
            lpb.row = host(lp["row"], np.int32)
            lpb.val = host(lp["val"], np.float64)
            lpb.c = host(lp["c"], np.float64)
        ctx = C.c_void_p()
        st = lib.sdp_setup_ex(C.byref(p), C.byref(spr) if spr is not None else None,
                              C.byref(lpb) if lpb is not None else None, C.byref(options),
                              _stream_ptr(self.stream), C.byref(ctx))
        if st != L.SDP_OK:
            raise SdpError(st, lib.sdp_last_error(None).decode())
        self._ctx = ctx

    # ---- lifecycle -----------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.sdp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != L.SDP_OK:
            raise SdpError(st, self._lib.sdp_last_error(self._ctx).decode())

    # ---- entry points --------------------------------------------------------------
    def aug_dim(self) -> int:
        v = self._lib.sdp_aug_dim(self._ctx)
        if v < 0:
            self._check(int(v))
        return int(v)

    def newton_apply(self, uv_in: torch.Tensor, uv_out: torch.Tensor | None = None, prec: int | None = None):
        """K [u; v] (eq. augsys); prec selects FP64 (default) or the context's low-precision form."""
        N = self.aug_dim()
        if uv_out is None:
            uv_out = torch.empty(N, dtype=torch.float64, device=uv_in.device)
        if prec is None:
            st = self._lib.sdp_newton_apply(self._ctx, _dptr(uv_in, "uv_in", N), _dptr(uv_out, "uv_out", N))
        else:
            st = self._lib.sdp_newton_apply_prec(self._ctx, int(prec), _dptr(uv_in, "uv_in", N),
                                                 _dptr(uv_out, "uv_out", N))
        self._check(st)
        return uv_out

    def precond_apply(self, uv_in: torch.Tensor, uv_out: torch.Tensor | None = None):
        """P^{-1} [f; h] with the Section 6 preconditioner (block elimination + one refinement step)."""
        N = self.aug_dim()
        if uv_out is None:
            uv_out = torch.empty(N, dtype=torch.float64, device=uv_in.device)
        st = self._lib.sdp_precond_apply(self._ctx, _dptr(uv_in, "uv_in", N), _dptr(uv_out, "uv_out", N))
        self._check(st)
        return uv_out

    def inner_solve(self, b_tilde: torch.Tensor, C_tilde: torch.Tensor, raise_on_notconv: bool = True):
        n, m = self.n, self.m
        dX = torch.empty((n, n), dtype=torch.float64, device=b_tilde.device)
        dy = torch.empty(m, dtype=torch.float64, device=b_tilde.device)
        s = L.SdpInnerStats()
        st = self._lib.sdp_inner_solve(self._ctx, _dptr(b_tilde, "b_tilde", m), _dptr(C_tilde, "C_tilde", n * n),
                                       _dptr(dX, "dX"), _dptr(dy, "dy"), C.byref(s))
        if st != L.SDP_OK and (raise_on_notconv or st != L.SDP_ENOTCONV):
            self._check(st)
        return dX, dy, L.struct_dict(s)

    def inner_solve_lp(self, b_tilde: torch.Tensor, C_tilde: torch.Tensor, c_tilde: torch.Tensor,
                       raise_on_notconv: bool = True):
        """Newton step with the LP block: (dX, dy, dx, stats)."""
        n, m, ell = self.n, self.m, self.ell
        dX = torch.empty((n, n), dtype=torch.float64, device=b_tilde.device)
        dy = torch.empty(m, dtype=torch.float64, device=b_tilde.device)
        dx = torch.empty(ell, dtype=torch.float64, device=b_tilde.device)
        s = L.SdpInnerStats()
        st = self._lib.sdp_inner_solve_lp(self._ctx, _dptr(b_tilde, "b_tilde", m), _dptr(C_tilde, "C_tilde", n * n),
                                          _dptr(c_tilde, "c_tilde", ell), _dptr(dX, "dX"), _dptr(dy, "dy"),
                                          _dptr(dx, "dx"), C.byref(s))
        if st != L.SDP_OK and (raise_on_notconv or st != L.SDP_ENOTCONV):
            self._check(st)
        return dX, dy, dx, L.struct_dict(s)

    def lp_split(self) -> dict:
        """The LP split at the current scaling: T (increasing) and w = sqrt(x/s)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        t = C.c_int32()
        cap = max(1, int(self.options.lp_top_max))
        top = torch.empty(cap, dtype=torch.int32, device=dev)
        w = torch.empty(self.ell, dtype=torch.float64, device=dev)
        self._check(self._lib.sdp_get_lp_split(self._ctx, C.byref(t), C.c_void_p(top.data_ptr()), _dptr(w, "w")))
        return {"t": t.value, "T": top[: t.value].clone(), "w": w}

    def adjoint(self, dL_dX: torch.Tensor, raise_off_centre: bool = True):
        """(dL/db, dL/dC, stats) for a loss gradient dL/dX at the current (re-centred) iterate.

        Raises SdpError(SDP_ECENTER) when the iterate could not be brought onto
        the central path, unless raise_off_centre is False (then stats["status"]
        says so and the outputs are the Newton-system solution at the iterate).
        """
        n, m = self.n, self.m
        G = dL_dX.detach().to(dtype=torch.float64).contiguous()
        gb = torch.empty(m, dtype=torch.float64, device=G.device)
        gC = torch.empty((n, n), dtype=torch.float64, device=G.device)
        s = L.SdpAdjointStats()
        st = self._lib.sdp_adjoint(self._ctx, _dptr(G, "dL_dX", n * n), _dptr(gb, "dL_db"), _dptr(gC, "dL_dC"),
                                   C.byref(s))
        if st != L.SDP_OK and (raise_off_centre or st != L.SDP_ECENTER):
            self._check(st)
        out = L.struct_dict(s)
        out["status"] = int(st)
        return gb, gC, out

    def ipm_step(self) -> dict:
        s = L.SdpStepStats()
        self._check(self._lib.sdp_ipm_step(self._ctx, C.byref(s)))
        return L.struct_dict(s)

    def solve(self, raise_on_stall: bool = True) -> dict:
        r = L.SdpResult()
        st = self._lib.sdp_solve(self._ctx, C.byref(r))
        if st != L.SDP_OK and (raise_on_stall or st != L.SDP_ESTALL):
            self._check(st)
        return L.struct_dict(r)

    def get_point(self):
        n, m = self.n, self.m
        dev = torch.device("cuda", torch.cuda.current_device())
        X = torch.empty((n, n), dtype=torch.float64, device=dev)
        y = torch.empty(m, dtype=torch.float64, device=dev)
        S = torch.empty((n, n), dtype=torch.float64, device=dev)
        self._check(self._lib.sdp_get_point(self._ctx, _dptr(X, "X"), _dptr(y, "y"), _dptr(S, "S")))
        return X, y, S

    def set_point(self, X: torch.Tensor, y: torch.Tensor, S: torch.Tensor, x: torch.Tensor | None = None,
                  s: torch.Tensor | None = None):
        """Replace the iterate; x and s (the LP block) are required exactly when the problem has one."""
        n, m = self.n, self.m
        if self.ell == 0:
            self._check(self._lib.sdp_set_point(self._ctx, _dptr(X, "X", n * n), _dptr(y, "y", m),
                                                _dptr(S, "S", n * n)))
        else:
            if x is None or s is None:
                raise ValueError("the problem has an LP block: pass x and s")
            self._check(self._lib.sdp_set_point_lp(self._ctx, _dptr(X, "X", n * n), _dptr(y, "y", m),
                                                   _dptr(S, "S", n * n), _dptr(x, "x", self.ell),
                                                   _dptr(s, "s", self.ell)))

    def get_lp_point(self):
        """(x, s) of the LP block."""
        dev = torch.device("cuda", torch.cuda.current_device())
        x = torch.empty(self.ell, dtype=torch.float64, device=dev)
        s = torch.empty(self.ell, dtype=torch.float64, device=dev)
        self._check(self._lib.sdp_get_point_lp(self._ctx, None, None, None, _dptr(x, "x"), _dptr(s, "s")))
        return x, s

    def get_scaling(self) -> dict:
        n = self.n
        lam = (C.c_double * n)()
        dev = torch.device("cuda", torch.cuda.current_device())
        V = torch.empty((n, n), dtype=torch.float64, device=dev)
        r = C.c_int32()
        tau = C.c_double()
        beta = C.c_double()
        self._check(self._lib.sdp_get_scaling(self._ctx, lam, _dptr(V, "V"), C.byref(r), C.byref(tau), C.byref(beta)))
        return {"lam": np.array(lam[:]), "V": V.T, "r": r.value, "tau": tau.value, "beta": beta.value}

    def profile_enable(self, classes=None):
        """Time the given kernel classes (iterable of SDP_K_*; None = all; [] = off)."""
        if classes is None:
            mask = (1 << L.SDP_K_COUNT) - 1
        else:
            mask = 0
            for k in classes:
                mask |= 1 << int(k)
        self._check(self._lib.sdp_profile_enable(self._ctx, mask))

    def profile_get(self, kernel_class: int) -> dict:
        ms = C.c_double()
        cnt = C.c_int64()
        by = C.c_double()
        self._check(self._lib.sdp_profile_get(self._ctx, kernel_class, C.byref(ms), C.byref(cnt), C.byref(by)))
        return {"ms": ms.value, "launches": cnt.value, "bytes": by.value}


def solve(problem: dict, **opts) -> tuple[dict, tuple]:
    """Set up, solve and return (result, (X, y, S))."""
    with Context(problem, **opts) as ctx:
        res = ctx.solve()
        return res, ctx.get_point()
