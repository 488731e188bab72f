"""Python binding of include/wcsdp_linalg.h (argument marshalling only).

Matrices are exchanged as column-major device buffers: an m x k matrix A is
held by a torch tensor of shape (k, m) whose rows are A's columns.  The
helpers ``to_dev`` / ``from_dev`` convert numpy (row, column) arrays.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .api import SdpError, _stream_ptr


def to_dev(a: np.ndarray) -> torch.Tensor:
    """Column-major device copy of a 2-D numpy array."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)).cuda()


def from_dev(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().T.copy()


def _p(t):
    if t is None:
        return C.c_void_p(0)
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _chk(st):
    if st != 0:
        raise SdpError(st, L.lib().sdp_last_error(None).decode())


def dsymv(alpha, A: torch.Tensor, x: torch.Tensor, beta=0.0, y: torch.Tensor | None = None):
    """y = alpha A x + beta y for a symmetric column-major A (d x d, as from to_dev), reading one triangle."""
    d = A.shape[0]
    lda = d + (d & 1)  # the kernel wants an even pitch
    Ap = A
    if lda != d:
        Ap = torch.zeros((d, lda), dtype=torch.float64, device=A.device)
        Ap[:, :d] = A
    if y is None:
        y = torch.zeros(d, dtype=torch.float64, device=A.device)
    _chk(L.lib().wc_dsymv(_stream_ptr(), d, alpha, _p(Ap), lda, _p(x), beta, _p(y)))
    return y


def dgemm(transa: str, transb: str, alpha, A: torch.Tensor, B: torch.Tensor, beta=0.0, Cm: torch.Tensor | None = None):
    """C = alpha op(A) op(B) + beta C on column-major device buffers (shapes as in to_dev)."""
    ka, ma = A.shape  # A is ma x ka column-major
    kb, mb = B.shape
    m = ka if transa == "T" else ma
    k = ma if transa == "T" else ka
    n = mb if transb == "T" else kb
    kk = kb if transb == "T" else mb
    assert k == kk, "inner dimensions differ"
    if Cm is None:
        Cm = torch.zeros((n, m), dtype=torch.float64, device=A.device)
    _chk(L.lib().wc_dgemm(_stream_ptr(), transa.encode(), transb.encode(), m, n, k, alpha, _p(A), ma, _p(B), mb, beta,
                          _p(Cm), m))
    return Cm


def dgemm_sym_lower(A: torch.Tensor, B: torch.Tensor, Cm: torch.Tensor | None = None):
    """The entries with row >= col of C = A B (n x n, column-major buffers as in to_dev), for products known
    to be symmetric; entries above the diagonal are left as they are or overwritten."""
    k, n = A.shape  # A is n x k column-major
    assert tuple(B.shape) == (n, k), "B must be k x n"
    if Cm is None:
        Cm = torch.zeros((n, n), dtype=torch.float64, device=A.device)
    _chk(L.lib().wc_dgemm_sym_lower(_stream_ptr(), n, k, _p(A), n, _p(B), k, _p(Cm), n))
    return Cm


def dpotrf(A: torch.Tensor):
    n = A.shape[0]
    info = C.c_int32()
    st = L.lib().wc_dpotrf(_stream_ptr(), n, _p(A), n, C.byref(info))
    return st, info.value


def dtrtri(Lm: torch.Tensor) -> torch.Tensor:
    n = Lm.shape[0]
    out = torch.empty_like(Lm)
    _chk(L.lib().wc_dtrtri(_stream_ptr(), n, _p(Lm), n, _p(out), n))
    return out


def dlanczos_min_eig(T: torch.Tensor, kmax: int = 64) -> float:
    n = T.shape[0]
    out = C.c_double()
    _chk(L.lib().wc_dlanczos_min_eig(_stream_ptr(), n, _p(T), n, kmax, C.byref(out)))
    return out.value


def djacobi_svd(A: torch.Tensor, want_v: bool = True, tol: float = 0.0, max_sweeps: int = 60):
    n = A.shape[0]
    V = torch.empty_like(A) if want_v else None
    s = torch.empty(n, dtype=torch.float64, device=A.device)
    sw = C.c_int32()
    _chk(L.lib().wc_djacobi_svd(_stream_ptr(), n, _p(A), n, _p(V), n, _p(s), tol, max_sweeps, C.byref(sw)))
    return s, V, sw.value


def _praw(t):
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


_LP_DTYPE = {1: torch.float32, 2: torch.int16}  # BF16 is carried as raw 16-bit patterns


def to_lowp(A: torch.Tensor, prec: int) -> torch.Tensor:
    """Column-major FP64 device matrix rounded to FP32 (prec 1) or BF16 bit patterns (prec 2)."""
    cols, rows = A.shape
    out = torch.empty((cols, rows), dtype=_LP_DTYPE[prec], device=A.device)
    _chk(L.lib().wc_to_lowp(_stream_ptr(), prec, rows, cols, _p(A), rows, _praw(out), rows))
    return out


def gemm_lp_sym(prec: int, out_kind: int, A: torch.Tensor, B: torch.Tensor, Cm: torch.Tensor | None = None):
    """C = A B for a symmetric A (m x m) and B (m x n) in precision prec, column-major as from to_lowp."""
    m, m2 = A.shape
    n, kb = B.shape
    assert m == m2 == kb, "A must be square and match B"
    if Cm is None:
        dt = {0: torch.float32, 1: torch.int16, 2: torch.float64, 3: torch.float64}[out_kind]
        Cm = torch.zeros((n, m), dtype=dt, device=A.device)
    _chk(L.lib().wc_gemm_lp_sym(_stream_ptr(), prec, out_kind, m, n, _praw(A), m, _praw(B), m, _praw(Cm), m))
    return Cm


def gemm_lp(prec: int, out_kind: int, A: torch.Tensor, B: torch.Tensor, Cm: torch.Tensor | None = None):
    """C = A B with low-precision column-major operands (as from to_lowp); out_kind 0 FP32, 1 BF16, 2 FP64 +=."""
    k, m = A.shape
    n, kb = B.shape
    assert k == kb, "inner dimensions differ"
    if Cm is None:
        dt = {0: torch.float32, 1: torch.int16, 2: torch.float64}[out_kind]
        Cm = torch.zeros((n, m), dtype=dt, device=A.device)
    _chk(L.lib().wc_gemm_lp(_stream_ptr(), prec, out_kind, m, n, k, _praw(A), m, _praw(B), k, _praw(Cm), m))
    return Cm
