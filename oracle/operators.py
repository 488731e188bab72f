"""The constraint operator A: S^n -> R^m and its adjoint (Introduction, eq. sdp-pd).

A(X)_i = <A_i, X> and A^T(y) = sum_i y_i A_i.  Three data forms:

* dense : problem["A"] is (m, n*n), row i = vec(A_i).
* entry : problem["jk"] is (m, 2), A_i = (e_j e_k^T + e_k e_j^T)/2, so
          A(X)_i = X_jk and A^T(y) places y_i/2 at (j,k) and (k,j)
          (y_i at (j,j) when j = k).
* sparse: problem["sp"] holds the entries of each A_i on and above the
          diagonal: constraint i owns ptr[i] .. ptr[i+1]-1 of (row, col, val)
          with row <= col, and A_i[row, col] = A_i[col, row] = val.

The matrix form used by the paper, script-A = [svec(A_1) ... svec(A_m)]^T
(Section 3), is built by ``amat`` for small instances.

A problem may also carry a nonnegative-orthant (LP) block x >= 0 entering
the constraints as A(X) + B x = b with cost c^T x (the cone of eq. rmc-sdp
and eq. snl-sdp).  problem["lp"] holds B column by column (compressed
sparse columns: ``ptr`` (l+1), ``row`` and ``val`` (nnz)) and ``c`` (l).
"""
from __future__ import annotations

import numpy as np

from .notation import svec, tri_len


def _sparse_owner(problem) -> np.ndarray:
    sp = problem["sp"]
    return np.repeat(np.arange(problem["m"]), np.diff(sp["ptr"]))


def a_op(problem, X: np.ndarray) -> np.ndarray:
    n = problem["n"]
    if problem["kind"] == "dense":
        return problem["A"] @ X.reshape(n * n)
    if problem["kind"] == "sparse":
        sp = problem["sp"]
        r, c, v = sp["row"], sp["col"], sp["val"]
        terms = v * np.where(r == c, X[r, c], X[r, c] + X[c, r])
        out = np.zeros(problem["m"])
        np.add.at(out, _sparse_owner(problem), terms)
        return out
    jk = problem["jk"]
    Xs = 0.5 * (X + X.T)
    return Xs[jk[:, 0], jk[:, 1]].copy()


def at_op(problem, y: np.ndarray) -> np.ndarray:
    n = problem["n"]
    if problem["kind"] == "dense":
        Y = (problem["A"].T @ y).reshape(n, n)
        return 0.5 * (Y + Y.T)
    if problem["kind"] == "sparse":
        sp = problem["sp"]
        r, c, v = sp["row"], sp["col"], sp["val"]
        w = v * y[_sparse_owner(problem)]
        Y = np.zeros((n, n))
        np.add.at(Y, (r, c), w)
        off = r != c
        np.add.at(Y, (c[off], r[off]), w[off])
        return Y
    jk = problem["jk"]
    Y = np.zeros((n, n))
    j = jk[:, 0]
    k = jk[:, 1]
    off = j != k
    np.add.at(Y, (j[off], k[off]), 0.5 * y[off])
    np.add.at(Y, (k[off], j[off]), 0.5 * y[off])
    np.add.at(Y, (j[~off], j[~off]), y[~off])
    return Y


def a_matrix(problem, i: int) -> np.ndarray:
    """The symmetric matrix A_i."""
    n = problem["n"]
    if problem["kind"] == "dense":
        return problem["A"][i].reshape(n, n).copy()
    if problem["kind"] == "sparse":
        sp = problem["sp"]
        M = np.zeros((n, n))
        for q in range(sp["ptr"][i], sp["ptr"][i + 1]):
            r, c, v = sp["row"][q], sp["col"][q], sp["val"][q]
            M[r, c] += v
            if r != c:
                M[c, r] += v
        return M
    j, k = problem["jk"][i]
    M = np.zeros((n, n))
    M[j, k] += 0.5
    M[k, j] += 0.5
    return M


def amat(problem) -> np.ndarray:
    """script-A = [svec(A_1), ..., svec(A_m)]^T, shape (m, n(n+1)/2)."""
    n = problem["n"]
    m = problem["m"]
    out = np.empty((m, tri_len(n)))
    for i in range(m):
        out[i] = svec(a_matrix(problem, i))
    return out


def frob_norms(problem) -> np.ndarray:
    """||A_i||_F for every constraint."""
    if problem["kind"] == "dense":
        return np.linalg.norm(problem["A"], axis=1)
    if problem["kind"] == "sparse":
        sp = problem["sp"]
        sq = sp["val"] ** 2 * np.where(sp["row"] == sp["col"], 1.0, 2.0)
        out = np.zeros(problem["m"])
        np.add.at(out, _sparse_owner(problem), sq)
        return np.sqrt(out)
    jk = problem["jk"]
    return np.where(jk[:, 0] == jk[:, 1], 1.0, np.sqrt(0.5))


def has_lp(problem) -> bool:
    return problem.get("lp") is not None


def lp_len(problem) -> int:
    return int(problem["lp"]["c"].size) if has_lp(problem) else 0


def b_matrix(problem) -> np.ndarray:
    """The dense m x l matrix B of the LP block, entry by entry from its columns (built once)."""
    lp = problem["lp"]
    if "_B" not in lp:
        ell = lp["c"].size
        B = np.zeros((problem["m"], ell))
        for j in range(ell):
            for q in range(lp["ptr"][j], lp["ptr"][j + 1]):
                B[lp["row"][q], j] += lp["val"][q]
        lp["_B"] = B
    return lp["_B"]


def b_op(problem, x: np.ndarray) -> np.ndarray:
    """B x."""
    return b_matrix(problem) @ x


def bt_op(problem, y: np.ndarray) -> np.ndarray:
    """B^T y."""
    return b_matrix(problem).T @ y
