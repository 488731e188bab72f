"""The seeded input generators (workloads/) do what their recipes say.

The full-size GPU checks on the n = 4000 completion workload take E in closed
form from `centred_pair`, so its guarantees are pinned here against the
definitions: a symmetric positive-definite pair with XS = mu I, whose
Nesterov-Todd scaling is V diag(sqrt(x/s)) V^T (the oracle's NT factor agrees)
and whose eigen-split picks the planted rank.  The completion and sensing
generators are checked for distinct, ordered pairs, b = A(X*) and symmetric
constraint matrices.
"""
import numpy as np
import pytest

import workloads
from oracle import nt, reform as rf


@pytest.mark.parametrize("n,r,mu", [(40, 3, 1e-2), (64, 4, 1e-6)])
def test_centred_pair_closed_form(n, r, mu):
    X, S, V, x, s = workloads.centred_pair(n, r, mu, seed=7)
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-12)
    assert np.array_equal(X, X.T) and np.array_equal(S, S.T)
    assert np.all(x > 0) and np.all(s > 0)
    assert np.allclose(x * s, mu, rtol=1e-14)
    # X S = mu I (perfect centrality)
    assert np.abs(X @ S - mu * np.eye(n)).max() <= 1e-9 * mu * n
    # the NT scaling point in closed form, against the oracle's factor (which
    # goes through Cholesky factors of X and S: accurate to about cond(X) eps)
    W = (V * np.sqrt(x / s)) @ V.T
    G, _, _ = nt.nt_factor(X, S)
    bound = 100 * (x.max() / x.min()) * np.finfo(float).eps
    assert np.abs(G @ G.T - W).max() <= bound * np.abs(W).max()
    # W S W = X, up to the rounding of the product (|W|^2 |S| eps per entry)
    wsw = 10 * n * np.finfo(float).eps * np.abs(W).max() ** 2 * np.abs(S).max()
    assert np.abs(W @ S @ W - X).max() <= wsw
    # the rank rule finds the r planted directions, and tau = lambda_{r+1} / 2
    sp = rf.eig_split(W, rank_max=10)
    lam = np.sort(np.sqrt(x / s))[::-1]
    assert sp["r"] == r
    assert abs(sp["tau"] - 0.5 * lam[r]) <= 1e-9 * lam[r]


def test_matrix_completion_pattern_and_values():
    p = workloads.matrix_completion(30, 2, 200, seed=5)
    jk = p["jk"]
    assert jk.shape == (200, 2) and jk.dtype == np.int32
    assert np.all(jk[:, 0] <= jk[:, 1]) and np.all(jk >= 0) and np.all(jk < 30)
    assert len({(int(a), int(b)) for a, b in jk}) == 200
    Xs = p["U"] @ p["U"].T
    assert np.allclose(p["b"], Xs[jk[:, 0], jk[:, 1]], rtol=1e-14, atol=0)
    assert np.array_equal(p["C"], np.eye(30))
    with pytest.raises(ValueError):
        workloads.matrix_completion(4, 1, 11, seed=0)  # more entries than n(n+1)/2


def test_gaussian_sensing_symmetric_and_planted():
    p = workloads.gaussian_sensing(8, 2, 20, seed=3)
    A = p["A"].reshape(20, 8, 8)
    assert np.array_equal(A, A.transpose(0, 2, 1))
    assert np.allclose(p["b"], np.einsum("ijk,jk->i", A, p["U"] @ p["U"].T), rtol=1e-12, atol=1e-14)
    assert p["kind"] == "dense"
