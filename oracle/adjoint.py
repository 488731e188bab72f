"""Gradient of a loss of the SDP solution with respect to the data (b, C).

Test infrastructure only (see oracle/__init__.py).

The paper does not treat derivatives; this follows from its Newton system
(Section 3, eq. Newt-eps).  At an interior iterate with Nesterov-Todd scaling
W, the Newton KKT operator

    K_N [dX; dy] = [ -W^{-1} dX W^{-1} + A^T(dy) ;  A(dX) ]

is self-adjoint, and the Newton direction of eq. Newt-eps with data (C~, b~)
is K_N^{-1} [C~; b~].  Perturbing the problem data by (dC, db) moves the
central-path point (A(X) = b, A^T(y) + S = C, XS = mu I) by the same kind of
system: A(dX) = db, A^T(dy) + dS = dC and, on the central path where
W = X / sqrt(mu), the NT linearisation dX + W dS W = 0 is exactly the
linearisation of XS = mu I.  So [dX; dy] = K_N^{-1} [dC; db], and for a loss
L(X) with gradient G_X,

    dL = <G_X, dX> = <K_N^{-1} [G_X; 0], [dC; db]>,

i.e. (dL/dC, dL/db) is the Newton direction with C~ = G_X and b~ = 0.  As
mu -> 0 this is the derivative of the solution map, for problems whose
solution map is differentiable (nondegenerate, strictly complementary).

The identity W = X / sqrt(mu) that makes the NT linearisation exact holds on
the central path only; an interior-point iterate sits in a neighbourhood of
it, and there the linearisation is off by a relative amount of the order of
the distance to the path (measured: 160 to 320 against 179 by finite
differences).  So the final iterate is first moved onto the central path at
its own mu by pure centring Newton steps (sigma = 1, no second-order term),
which converge quadratically.
"""
from __future__ import annotations

import numpy as np

from . import ipm
from .notation import sym
from .nt import nt_factor


def kkt_gradient(problem, X, S, GX):
    """(dL/dC, dL/db) at the iterate (X, S) for a loss with gradient GX, by the direct Newton solve."""
    n, m = problem["n"], problem["m"]
    G, _, _ = nt_factor(X, S)
    W = G @ G.T
    fac = ipm.schur_factor(problem, G, W)
    dX, dy, _ = ipm.newton_direct(problem, G, fac, np.zeros(m), sym(np.asarray(GX, dtype=float)), np.zeros((n, n)))
    return dX, dy


def center(problem, X, y, S, mu=None, tol=1e-8, maxit=12):
    """Newton steps towards the central-path point (A(X) = b, A^T(y) + S = C, XS = mu I).

    NT direction of eq. Newt-eps with b~ = r_p and C~ = R_d - G^{-T} H G^{-1},
    H = diag((mu - d_i^2) / d_i) (the corrector's H with sigma mu = mu and no
    second-order term); step min(1, 0.95 alpha_max) for both X and S.  The
    distance to the point is max(||d^2 / mu - 1||, pinf, dinf) (d^2 are the
    eigenvalues of XS; pinf, dinf the relative infeasibilities).  Stops when it
    is <= tol, or when two steps in a row fail to reduce it by 10% (rounding
    floor, or no central path: without a strictly feasible point the iterates
    drift off instead); returns the closest point seen.
    """
    n = problem["n"]
    if mu is None:
        mu = float(np.sum(X * S)) / n
    best = (np.inf, X, y, S)
    stall = 0
    for _ in range(maxit):
        r = ipm.residuals(problem, X, y, S)
        G, d, _ = nt_factor(X, S)
        dev = max(np.linalg.norm(d ** 2 / mu - 1.0), r["pinf"], r["dinf"])
        stall = stall + 1 if dev > 0.9 * best[0] else 0
        if dev < best[0]:
            best = (dev, X, y, S)
        if dev <= tol or stall >= 2:
            break
        W = G @ G.T
        Gi = np.linalg.inv(G)
        H = np.diag((mu - d ** 2) / d)
        Ct = r["Rd"] - Gi.T @ H @ Gi
        dX, dy, dS = ipm.newton_direct(problem, G, ipm.schur_factor(problem, G, W), r["rp"], Ct, r["Rd"])
        a = min(1.0, 0.95 * ipm.max_step(np.linalg.cholesky(X), dX), 0.95 * ipm.max_step(np.linalg.cholesky(S), dS))
        while True:  # the eigenvalue bound is exact only up to rounding: confirm both stay PD
            try:
                np.linalg.cholesky(sym(X + a * dX))
                np.linalg.cholesky(sym(S + a * dS))
                break
            except np.linalg.LinAlgError:
                a *= 0.5
        X, y, S = sym(X + a * dX), y + a * dy, sym(S + a * dS)
    else:
        r = ipm.residuals(problem, X, y, S)
        G, d, _ = nt_factor(X, S)
        dev = max(np.linalg.norm(d ** 2 / mu - 1.0), r["pinf"], r["dinf"])
        if dev < best[0]:
            best = (dev, X, y, S)
    return best[1], best[2], best[3]


def solution_gradient(problem, X, y, S, GX):
    """(dL/dC, dL/db) of the central-path point at the iterate's mu: centre, then kkt_gradient."""
    Xc, yc, Sc = center(problem, X, y, S)
    return kkt_gradient(problem, Xc, Sc, GX)


def perturbed(problem, db, dC, h):
    """The problem with b + h db and C + h dC."""
    q = dict(problem)
    q["b"] = problem["b"] + h * db
    q["C"] = problem["C"] + h * sym(dC)
    return q


def fd_directional(problem, loss, db, dC, h=1e-6, tol=1e-11):
    """Central difference (L(X(b + h db, C + h dC)) - L(X(b - h db, C - h dC))) / 2h of oracle solves."""
    lp = loss(ipm.solve(perturbed(problem, db, dC, h), tol=tol)["X"])
    lm = loss(ipm.solve(perturbed(problem, db, dC, -h), tol=tol)["X"])
    return (lp - lm) / (2.0 * h)
