"""Nesterov-Todd scaling point (Introduction, eq. newt).

The paper defines W = X^{1/2} (X^{1/2} S X^{1/2})^{-1/2} X^{1/2}, the unique
positive definite matrix with W S W = X.  ``nt_definition`` evaluates that
formula literally with symmetric matrix functions.  ``nt_factor`` gives the
factored form used by the interior-point iterations: with X = L L^T,
S = R R^T and the SVD R^T L = U D V^T, the matrix G = L V D^{-1/2}
satisfies W = G G^T and G^{-1} X G^{-T} = G^T S G = D (Todd, Toh and
Tutuncu's construction of the NT scaling).
"""
from __future__ import annotations

import numpy as np


def _sym_fun(M: np.ndarray, f) -> np.ndarray:
    w, V = np.linalg.eigh(0.5 * (M + M.T))
    return (V * f(w)) @ V.T


def nt_definition(X: np.ndarray, S: np.ndarray) -> np.ndarray:
    Xh = _sym_fun(X, np.sqrt)
    inner = _sym_fun(Xh @ S @ Xh, lambda w: 1.0 / np.sqrt(w))
    W = Xh @ inner @ Xh
    return 0.5 * (W + W.T)


def nt_factor(X: np.ndarray, S: np.ndarray):
    """Return (G, d, L) with W = G G^T, G^T S G = G^{-1} X G^{-T} = diag(d)."""
    L = np.linalg.cholesky(0.5 * (X + X.T))
    R = np.linalg.cholesky(0.5 * (S + S.T))
    _, d, Vt = np.linalg.svd(R.T @ L)
    G = (L @ Vt.T) / np.sqrt(d)
    return G, d, L
