"""Pins for the oracle's sparse constraint kind (entries of each A_i on and above the diagonal).

* A(X)_i = <A_i, X> and A^T(y) = sum_i y_i A_i against the matrices A_i
  written out entry by entry, adjointness <A(X), y> = <X, A^T(y)>, and
  ||A_i||_F;
* the same SNL instance (eq. snl-sdp) stored densely and sparsely gives the
  same interior-point solution.
"""
import numpy as np

import workloads
from oracle import ipm, operators as ops


def snl(kind):
    return workloads.sensor_localization(12, 50, 20, 2, 1, seed=4, kind=kind)


def test_sparse_operators_match_definition():
    p = snl("sparse")
    n, m = p["n"], p["m"]
    rng = np.random.default_rng(1)
    X = rng.standard_normal((n, n))  # not symmetric: <A_i, X> uses both triangles
    y = rng.standard_normal(m)
    A = [np.zeros((n, n)) for _ in range(m)]
    sp = p["sp"]
    for i in range(m):
        for q in range(sp["ptr"][i], sp["ptr"][i + 1]):
            r, c, v = sp["row"][q], sp["col"][q], sp["val"][q]
            assert r <= c
            A[i][r, c] = v
            A[i][c, r] = v
    ax = np.array([np.sum(Ai * X) for Ai in A])
    assert np.allclose(ops.a_op(p, X), ax, rtol=1e-14, atol=1e-13)
    assert np.allclose(ops.at_op(p, y), sum(yi * Ai for yi, Ai in zip(y, A)), rtol=1e-14, atol=1e-13)
    Xs = 0.5 * (X + X.T)
    assert abs(ops.a_op(p, Xs) @ y - np.sum(Xs * ops.at_op(p, y))) <= 1e-12 * np.abs(ax).sum()
    assert np.allclose(ops.frob_norms(p), [np.linalg.norm(Ai) for Ai in A], rtol=1e-15)
    for i in (0, 3, m - 1):
        assert np.array_equal(ops.a_matrix(p, i), A[i])


def test_sparse_and_dense_snl_solve_identically():
    pd, ps = snl("dense"), snl("sparse")
    assert np.array_equal(pd["b"], ps["b"])
    rd, rs = ipm.solve(pd), ipm.solve(ps)
    assert rd["status"] == rs["status"] == "converged"
    assert rd["iterations"] == rs["iterations"]
    assert np.linalg.norm(rd["X"] - rs["X"]) <= 1e-9 * np.linalg.norm(rd["X"])
    d = ps["d"]
    assert np.linalg.norm(rs["X"][:d, d:] - ps["Ystar"]) <= 1e-6
