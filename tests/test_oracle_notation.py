"""Pins for the oracle's notation, constraint operators and NT scaling."""
import numpy as np
import pytest

import workloads
from oracle import notation as nt_
from oracle import nt, operators as ops


def rand_sym(n, rng):
    M = rng.standard_normal((n, n))
    return 0.5 * (M + M.T)


def test_svec_inner_product_and_inverse():
    # Notations: <X, S> = svec(X)^T svec(S) for symmetric X, S; smat inverts svec.
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 9):
        X, S = rand_sym(n, rng), rand_sym(n, rng)
        assert np.isclose(nt_.svec(X) @ nt_.svec(S), np.trace(X @ S), rtol=1e-13, atol=1e-13)
        assert np.allclose(nt_.smat(nt_.svec(X), n), X, atol=1e-15)
        assert nt_.svec(X).size == n * (n + 1) // 2


def test_svec_order_matches_definition():
    # svec = [X11, sqrt2 X21, ..., sqrt2 Xn1, X22, sqrt2 X32, ..., Xnn].
    X = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 5.0], [3.0, 5.0, 6.0]])
    s2 = np.sqrt(2.0)
    assert np.allclose(nt_.svec(X), [1.0, 2 * s2, 3 * s2, 4.0, 5 * s2, 6.0])


def test_psi_basis():
    rng = np.random.default_rng(1)
    n = 4
    P = nt_.psi(n)
    X = rand_sym(n, rng)
    assert np.allclose(P.T @ nt_.vec(X), nt_.svec(X))
    assert np.allclose(P @ nt_.svec(X), nt_.vec(X))
    assert np.allclose(P.T @ P, np.eye(n * (n + 1) // 2))


def test_symmetric_kronecker_action():
    # (A (x)_s B) svec(X) = (B (x)_s A) svec(X) = svec(A X B^T) for X in S^r.
    rng = np.random.default_rng(2)
    n, r = 5, 3
    A = rng.standard_normal((n, r))
    B = rng.standard_normal((n, r))
    X = rand_sym(r, rng)
    lhs = nt_.skron(A, B) @ nt_.svec(X)
    assert np.allclose(lhs, nt_.svec(A @ X @ B.T), atol=1e-13)
    assert np.allclose(nt_.skron(B, A) @ nt_.svec(X), lhs, atol=1e-13)


@pytest.mark.parametrize("kind", ["dense", "entry"])
def test_operator_adjoint_and_matrix_form(kind):
    rng = np.random.default_rng(3)
    if kind == "dense":
        p = workloads.gaussian_sensing(6, 2, 12, seed=5)
    else:
        p = workloads.matrix_completion(6, 2, 15, seed=5)
    X = rand_sym(6, rng)
    y = rng.standard_normal(p["m"])
    # <A(X), y> = <X, A^T(y)>
    assert np.isclose(ops.a_op(p, X) @ y, np.sum(X * ops.at_op(p, y)), rtol=1e-13)
    # A(X) = script-A svec(X)
    assert np.allclose(ops.amat(p) @ nt_.svec(X), ops.a_op(p, X), atol=1e-13)
    if kind == "entry":
        jk = p["jk"]
        assert np.allclose(ops.a_op(p, X), X[jk[:, 0], jk[:, 1]])
        assert np.all(jk[:, 0] <= jk[:, 1])
        assert len({tuple(t) for t in jk}) == p["m"]


def test_planted_measurements():
    p = workloads.gaussian_sensing(7, 2, 20, seed=9)
    Xs = p["U"] @ p["U"].T
    assert np.allclose(ops.a_op(p, Xs), p["b"])
    q = workloads.matrix_completion(7, 2, 20, seed=9)
    Xq = q["U"] @ q["U"].T
    assert np.allclose(ops.a_op(q, Xq), q["b"])


def test_nt_scaling_definition_and_factor():
    # eq. newt: W = X^{1/2}(X^{1/2} S X^{1/2})^{-1/2} X^{1/2} is the PD matrix with W S W = X.
    for seed in range(3):
        X, S = workloads.random_pd_pair(6, seed, spread=1.5)
        W = nt.nt_definition(X, S)
        assert np.allclose(W @ S @ W, X, rtol=1e-10, atol=1e-10 * np.linalg.norm(X))
        assert np.linalg.eigvalsh(W)[0] > 0
        # the second expression of eq. newt
        def mf(M, f):
            w, V = np.linalg.eigh(M)
            return (V * f(w)) @ V.T
        Sh = mf(S, np.sqrt)
        W2 = np.linalg.inv(Sh @ mf(Sh @ X @ Sh, lambda w: 1 / np.sqrt(w)) @ Sh)
        assert np.allclose(W, W2, rtol=1e-9, atol=1e-9 * np.linalg.norm(W))
        G, d, L = nt.nt_factor(X, S)
        assert np.allclose(G @ G.T, W, rtol=1e-9, atol=1e-9 * np.linalg.norm(W))
        assert np.allclose(G.T @ S @ G, np.diag(d), atol=1e-9 * d.max())
        Gi = np.linalg.inv(G)
        assert np.allclose(Gi @ X @ Gi.T, np.diag(d), atol=1e-9 * d.max())
