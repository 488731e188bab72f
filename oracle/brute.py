"""Tiny SDP instances whose optimum is known without an interior-point method.

* ``lp_instance`` / ``lp_optimum``: with diagonal A_i = diag(a_i) and
  C = diag(c) the SDP of eq. sdp-pd reduces to the linear program
  min c^T x s.t. a_i^T x = b_i, x >= 0 on x = diag(X) (off-diagonal entries of X
  enter neither the objective nor the constraints, and diag(x) is PSD exactly
  when x >= 0).  Its optimum is found by enumerating every basic solution.
* ``two_by_two_optimum``: n = 2 with m = 2 constraints leaves a line
  X(t) = X0 + t D of feasible symmetric matrices; X(t) is PSD on the interval
  where trace >= 0 and det X(t) >= 0, a quadratic in t, so the linear
  objective is optimal at one of that quadratic's roots.
* ``determined_instance``: m = n(n+1)/2 linearly independent constraints fix
  X = smat(script-A^{-1} b); when that X is PSD it is the unique feasible
  point and hence optimal.
"""
from __future__ import annotations

import itertools

import numpy as np

from .notation import smat, svec


def lp_instance(n: int, m: int, seed: int):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 2.0, size=(m, n))
    x_feas = rng.uniform(0.5, 1.5, size=n)
    b = a @ x_feas
    c = rng.uniform(0.5, 2.0, size=n)
    A = np.stack([np.diag(a[i]).reshape(-1) for i in range(m)])
    return {"kind": "dense", "n": n, "m": m, "A": A, "b": b, "C": np.diag(c), "lp_data": (a, b, c)}


def lp_optimum(a: np.ndarray, b: np.ndarray, c: np.ndarray):
    m, n = a.shape
    best = (np.inf, None)
    for cols in itertools.combinations(range(n), m):
        B = a[:, cols]
        if abs(np.linalg.det(B)) < 1e-12:
            continue
        xb = np.linalg.solve(B, b)
        if np.all(xb >= -1e-12):
            x = np.zeros(n)
            x[list(cols)] = xb
            val = float(c @ x)
            if val < best[0]:
                best = (val, x)
    return best


def two_by_two_instance(seed: int):
    """n = 2, m = 2 with a strictly feasible point and a PD cost."""
    rng = np.random.default_rng(seed)
    X0 = np.array([[2.0, 0.3], [0.3, 1.5]])
    mats = []
    for _ in range(2):
        M = rng.standard_normal((2, 2))
        mats.append(0.5 * (M + M.T))
    b = np.array([np.sum(Mi * X0) for Mi in mats])
    Cm = rng.standard_normal((2, 2))
    C = Cm @ Cm.T + 0.5 * np.eye(2)
    A = np.stack([Mi.reshape(-1) for Mi in mats])
    return {"kind": "dense", "n": 2, "m": 2, "A": A, "b": b, "C": C, "X0": X0}


def two_by_two_optimum(problem):
    """Optimum of the n = 2, m = 2 instance from the roots of det X(t) = 0."""
    A = problem["A"]
    b = problem["b"]
    C = problem["C"]
    # coordinates x = (X11, X21, X22); <A_i, X> = A11 x1 + 2 A21 x2 + A22 x3
    rows = np.array([[Ai[0], 2.0 * Ai[1], Ai[3]] for Ai in A])
    # particular solution and null direction of the 2 x 3 system
    xp = np.linalg.lstsq(rows, b, rcond=None)[0]
    _, _, Vt = np.linalg.svd(rows)
    dvec = Vt[-1]

    def X_of(t):
        x = xp + t * dvec
        return np.array([[x[0], x[1]], [x[1], x[2]]])

    # det X(t) = (p1 + t d1)(p3 + t d3) - (p2 + t d2)^2 = qa t^2 + qb t + qc
    qa = dvec[0] * dvec[2] - dvec[1] ** 2
    qb = xp[0] * dvec[2] + xp[2] * dvec[0] - 2.0 * xp[1] * dvec[1]
    qc = xp[0] * xp[2] - xp[1] ** 2
    roots = np.roots([qa, qb, qc]) if abs(qa) > 1e-14 else np.array([-qc / qb])
    roots = np.real(roots[np.abs(np.imag(roots)) < 1e-12])
    cands = []
    for t in roots:
        Xt = X_of(t)
        if np.trace(Xt) >= 0:
            cands.append((float(np.sum(C * Xt)), Xt))
    val, Xopt = min(cands, key=lambda z: z[0])
    return val, Xopt


def determined_instance(n: int, seed: int):
    """m = n(n+1)/2 Gaussian constraints with a PD planted point."""
    rng = np.random.default_rng(seed)
    m = n * (n + 1) // 2
    G = rng.standard_normal((m, n, n)) / n
    A = 0.5 * (G + G.transpose(0, 2, 1))
    Mx = rng.standard_normal((n, n))
    X0 = Mx @ Mx.T + n * np.eye(n)
    Am = A.reshape(m, n * n)
    b = Am @ X0.reshape(-1)
    Cm = rng.standard_normal((n, n))
    C = Cm @ Cm.T + np.eye(n)
    return {"kind": "dense", "n": n, "m": m, "A": Am, "b": b, "C": C, "X0": X0}


def determined_optimum(problem):
    n, m = problem["n"], problem["m"]
    rows = np.stack([svec(problem["A"][i].reshape(n, n)) for i in range(m)])
    return smat(np.linalg.solve(rows, problem["b"]), n)
