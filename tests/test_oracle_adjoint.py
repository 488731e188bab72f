"""Pins of the oracle's KKT gradient (oracle/adjoint.py) against facts independent of it.

* LP closed form: with diagonal A_i and C the SDP is an LP in diag(X); at a
  nondegenerate vertex x_B = a_B^{-1} b, so for L = g^T x the gradient in b
  is a_B^{-T} g_B.  (dL/dC tends to zero there, but the direct formula
  dX = W (A^T dy - C~) W evaluates it as W^2 times a difference of O(1)
  terms, so at mu ~ 1e-11 its rounding error, ~eps / mu, is what a check
  would see; dL/dC is pinned by the envelope and finite-difference tests.)
* Envelope theorem: for L(X) = <C0, X> with C0 the problem's own C, the
  optimal value's sensitivity gives dL/db = y* and dL/dC = 0.
* Central finite differences (step 1e-6) of full solves to a 1e-11 gap, in
  random joint (db, dC) directions.
* Central finite differences (step 1e-7) of central-path points at a fixed
  mu, which exist whenever both problems are strictly feasible -- also for
  the planted, primal-degenerate sensing workload (n = 20, m = 120).

The last two need a differentiable solution map, i.e. a nondegenerate,
strictly complementary problem: generic data (workloads.generic_*).  The
planted low-rank workloads with m above the tangent dimension n r - r(r-1)/2
are primal degenerate (y* is not unique), and there the optimal value is
not differentiable in b.

The gradient is that of the central-path point at the final iterate's mu
(the iterate is re-centred first); the checks take it at a 1e-9 gap, where
the direct formula's rounding (~eps / mu) is still small.
"""
import numpy as np
import pytest

import workloads
from oracle import adjoint, brute, ipm


def test_lp_vertex_gradient_closed_form():
    # the seed gives a nondegenerate optimal vertex (checked below)
    q = brute.lp_instance(5, 2, 3)
    a, b, c = q["lp_data"]
    val, x = brute.lp_optimum(a, b, c)
    basis = np.flatnonzero(x > 1e-9)
    assert basis.size == q["m"]
    res = ipm.solve(q, tol=1e-11)
    g = np.random.default_rng(0).standard_normal(q["n"])
    gC, gb = adjoint.solution_gradient(q, res["X"], res["y"], res["S"], np.diag(g))
    expect = np.linalg.solve(a[:, basis].T, g[basis])
    e_b = np.abs(gb - expect).max() / np.abs(expect).max()
    assert e_b <= 1e-6


def generic(which):
    return workloads.generic_sensing(12, 30, seed=5) if which == "dense" else workloads.generic_completion(12, 30, seed=6)


@pytest.mark.parametrize("which", ["dense", "entry"])
def test_envelope_theorem(which):
    p = generic(which)
    res = ipm.solve(p, tol=1e-9)
    gC, gb = adjoint.solution_gradient(p, res["X"], res["y"], res["S"], p["C"])
    e_b = np.linalg.norm(gb - res["y"]) / np.linalg.norm(res["y"])
    assert e_b <= 5e-5
    assert np.linalg.norm(gC) <= 5e-5 * np.linalg.norm(res["X"])


@pytest.mark.parametrize("which", ["dense", "entry"])
def test_kkt_gradient_matches_finite_differences(which):
    p = generic(which)
    n, m = p["n"], p["m"]
    rng = np.random.default_rng(11)
    V = rng.standard_normal((n, 2))
    target = V @ V.T

    def loss(X):
        return float(np.sum((X - target) ** 2))

    res = ipm.solve(p, tol=1e-9)
    gC, gb = adjoint.solution_gradient(p, res["X"], res["y"], res["S"], 2.0 * (res["X"] - target))
    for k in range(3):
        db = rng.standard_normal(m)
        M = rng.standard_normal((n, n))
        dC = 0.5 * (M + M.T)
        fd = adjoint.fd_directional(p, loss, db, dC)
        an = float(gb @ db + np.sum(gC * dC))
        # the central-path derivative at mu ~ 1e-9 vs the solution map's:
        # measured differences 1e-5 .. 2e-4 relative on these instances
        assert abs(an - fd) <= 5e-4 * max(abs(fd), 1e-8), (k, an, fd)


def test_kkt_gradient_is_the_central_path_derivative():
    p = workloads.config(0)
    n, m = p["n"], p["m"]
    res = ipm.solve(p, tol=1e-2)
    mu = float(np.sum(res["X"] * res["S"])) / n
    Xc, yc, Sc = adjoint.center(p, res["X"], res["y"], res["S"], mu=mu, tol=1e-13, maxit=40)
    target = np.random.default_rng(11).standard_normal((n, 2))
    target = target @ target.T

    def loss(X):
        return float(np.sum((X - target) ** 2))

    gC, gb = adjoint.kkt_gradient(p, Xc, Sc, 2.0 * (Xc - target))
    rng = np.random.default_rng(3)
    h = 1e-7
    for k in range(2):
        db = rng.standard_normal(m)
        M = rng.standard_normal((n, n))
        dC = 0.5 * (M + M.T)
        Xp = adjoint.center(adjoint.perturbed(p, db, dC, h), Xc, yc, Sc, mu=mu, tol=1e-13, maxit=40)[0]
        Xm = adjoint.center(adjoint.perturbed(p, db, dC, -h), Xc, yc, Sc, mu=mu, tol=1e-13, maxit=40)[0]
        fd = (loss(Xp) - loss(Xm)) / (2 * h)
        an = float(gb @ db + np.sum(gC * dC))
        assert abs(an - fd) <= 1e-5 * abs(fd), (k, an, fd)
