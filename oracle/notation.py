"""Symmetric vectorisation and the symmetric Kronecker product (Notations).

svec(X) stacks the lower triangle of X column by column, multiplying the
off-diagonal entries by sqrt(2), so that <X, S> = svec(X)^T svec(S).
Psi_n is the n^2 x n(n+1)/2 basis of vec(S^n) with svec(X) = Psi_n^T vec(X)
for symmetric X.  For a non-symmetric argument svec(M) = svec((M+M^T)/2)
(Appendix A).  The symmetric Kronecker product of A, B in R^{n x r} is
A (x)_s B = 1/2 Psi_n^T (A (x) B + B (x) A) Psi_r.
"""
from __future__ import annotations

import numpy as np

SQRT2 = np.sqrt(2.0)


def tri_len(n: int) -> int:
    return n * (n + 1) // 2


def svec(X: np.ndarray) -> np.ndarray:
    """Column-major lower triangle of sym(X), off-diagonals times sqrt(2)."""
    n = X.shape[0]
    Xs = 0.5 * (X + X.T)
    out = np.empty(tri_len(n))
    p = 0
    for k in range(n):
        col = Xs[k:, k].copy()
        col[1:] *= SQRT2
        out[p : p + n - k] = col
        p += n - k
    return out


def smat(x: np.ndarray, n: int) -> np.ndarray:
    """Inverse of svec."""
    X = np.zeros((n, n))
    p = 0
    for k in range(n):
        col = x[p : p + n - k].copy()
        col[1:] /= SQRT2
        X[k:, k] = col
        X[k, k:] = col
        p += n - k
    return X


def psi(n: int) -> np.ndarray:
    """Psi_n: columns are vec of the symmetric basis matrices matching svec.

    Column for the diagonal position (k, k) is vec(e_k e_k^T); for the
    off-diagonal position (j, k), j > k, it is vec(e_j e_k^T + e_k e_j^T)/sqrt(2).
    Then Psi_n^T vec(X) = svec(X) and Psi_n svec(X) = vec(X) for symmetric X.
    """
    P = np.zeros((n * n, tri_len(n)))
    p = 0
    for k in range(n):
        for j in range(k, n):
            if j == k:
                P[k + n * k, p] = 1.0
            else:
                P[j + n * k, p] = 1.0 / SQRT2
                P[k + n * j, p] = 1.0 / SQRT2
            p += 1
    return P


def vec(X: np.ndarray) -> np.ndarray:
    """Column-stacking vectorisation."""
    return X.reshape(-1, order="F")


def skron(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A (x)_s B = 1/2 Psi_n^T (A (x) B + B (x) A) Psi_r for A, B in R^{n x r}."""
    n, r = A.shape
    Pn = psi(n)
    Pr = psi(r)
    return 0.5 * Pn.T @ (np.kron(A, B) + np.kron(B, A)) @ Pr


def sym(M: np.ndarray) -> np.ndarray:
    return 0.5 * (M + M.T)
