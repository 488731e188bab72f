"""Plain FP64 primal-dual interior-point method with direct Newton solves.

This is the textbook method the paper accelerates: each Newton subproblem
(Introduction, eq. newt; Section 3, eq. Newt-eps) is solved directly by
forming and factoring the m x m Schur complement M_ij = <A_i, W A_j W>,
which the Introduction names as the standard direct approach.  The outer
loop is an infeasible primal-dual path-following method with the
Nesterov-Todd direction and a Mehrotra predictor-corrector; the paper uses
SeDuMi for this loop and does not spell it out, so both the oracle and the
GPU library follow the same written-out algorithm (coded separately):

1. X = xi I, S = eta I, y = 0 (SDPT3-style magnitudes).
2. r_p = b - A(X), R_d = C - A^T(y) - S, mu = <X, S>/n; stop when the
   relative gap, primal and dual infeasibility are all <= tol.
3. NT factor G (oracle.nt.nt_factor), W = G G^T, d = diag(G^T S G).
4. Predictor: Newton system with b~ = r_p, C~ = R_d + S.
5. Step to the boundary of the PSD cone for X and S separately; sigma =
   (mu_aff / mu)^3.
6. Corrector: H_ij = [2(sigma mu - d_i^2) delta_ij - (Dx Ds + Ds Dx)_ij]/(d_i+d_j)
   with Dx = G^{-1} dX_a G^{-T}, Ds = G^T dS_a G; C~ = R_d - G^{-T} H G^{-1}.
7. Step lengths min(1, 0.98 alpha_max), update, repeat.

In every Newton system dX = W (A^T(dy) - C~) W and dS = R_d - A^T(dy), i.e.
the KKT system of eq. Newt-eps with the residual-form dS.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import operators as ops
from .nt import nt_factor
from .notation import sym


def start_point(problem):
    """xi, eta for X0 = xi I and S0 = eta I."""
    n = problem["n"]
    fn = ops.frob_norms(problem)
    b = problem["b"]
    xi = max(10.0, np.sqrt(n), n * float(np.max((1.0 + np.abs(b)) / (1.0 + fn))))
    eta = max(10.0, np.sqrt(n), 1.0 + max(float(np.max(fn)), float(np.linalg.norm(problem["C"]))))
    return xi, eta


def scaled_rows(problem, G: np.ndarray) -> np.ndarray:
    """Rows svec(G^T A_i G), so that M = A~ A~^T with M_ij = <A_i, W A_j W>."""
    n, m = problem["n"], problem["m"]
    jj, kk = np.tril_indices(n)
    w = np.where(jj == kk, 1.0, np.sqrt(2.0))
    if problem["kind"] == "dense":
        A = problem["A"].reshape(m, n, n)
        At = np.matmul(np.matmul(G.T[None], A), G[None])
    else:
        jk = problem["jk"]
        Gj = G[jk[:, 0]]
        Gk = G[jk[:, 1]]
        At = 0.5 * (Gj[:, :, None] * Gk[:, None, :] + Gk[:, :, None] * Gj[:, None, :])
    return At[:, jj, kk] * w


def schur_matrix(problem, G: np.ndarray, W: np.ndarray) -> np.ndarray:
    """M_ij = <A_i, W A_j W> formed explicitly."""
    if problem["kind"] == "dense":
        Ap = scaled_rows(problem, G)
        return Ap @ Ap.T
    jk = problem["jk"]
    j, k = jk[:, 0], jk[:, 1]
    return 0.5 * (W[np.ix_(j, j)] * W[np.ix_(k, k)] + W[np.ix_(j, k)] * W[np.ix_(k, j)])


def schur_factor(problem, G: np.ndarray, W: np.ndarray):
    """Thin QR of A~^T (rows svec(G^T A_i G)): A~^T = Q1 R, so M = R^T R.

    Factoring A~ instead of M avoids squaring the condition number; M itself
    becomes too ill-conditioned for a Cholesky factorisation as mu -> 0,
    which is the difficulty the Introduction attributes to the direct
    approach.
    """
    Ap = scaled_rows(problem, G)
    Q1, R = np.linalg.qr(Ap.T, mode="reduced")
    return Ap, Q1, R


def newton_direct(problem, G, fac, bt, Ct, Rd):
    """Direct solve of eq. Newt-eps in NT-scaled coordinates.

    With dX = G Z G^T the Newton subproblem (eq. newt) becomes
    min 1/2 ||z||^2 + cbar^T z  s.t.  A~ z = b~, where z = svec(Z) and
    cbar = svec(G^T C~ G); its KKT conditions are z = A~^T dy - cbar and
    A~ A~^T dy = b~ + A~ cbar, i.e. M dy = b~ + A(W C~ W) with
    dX = W (A^T(dy) - C~) W.  With A~^T = Q1 R: w = R^{-T}(b~ + A~ cbar),
    A~^T dy = Q1 w and dy = R^{-1} w.
    """
    Ap, Q1, R = fac
    n = problem["n"]
    jj, kk = np.tril_indices(n)
    wts = np.where(jj == kk, 1.0, np.sqrt(2.0))
    GCG = G.T @ Ct @ G
    cbar = GCG[jj, kk] * wts
    w = sla.solve_triangular(R, bt + Ap @ cbar, trans="T")
    dy = sla.solve_triangular(R, w)
    z = Q1 @ w - cbar
    Z = np.zeros((n, n))
    Z[jj, kk] = z / wts
    Z[kk, jj] = z / wts
    dX = sym(G @ Z @ G.T)
    dS = sym(Rd - ops.at_op(problem, dy))
    return dX, dy, dS


def max_step(L: np.ndarray, D: np.ndarray) -> float:
    """Largest alpha with L L^T + alpha D PSD: 1 / max(0, -lambda_min(L^{-1} D L^{-T}))."""
    T = sla.solve_triangular(L, D, lower=True)
    T = sla.solve_triangular(L, T.T, lower=True)
    lmin = float(np.linalg.eigvalsh(sym(T))[0])
    return np.inf if lmin >= 0 else -1.0 / lmin


def residuals(problem, X, y, S):
    b, C = problem["b"], problem["C"]
    rp = b - ops.a_op(problem, X)
    Rd = sym(C - ops.at_op(problem, y) - S)
    pobj = float(np.sum(C * X))
    dobj = float(b @ y)
    n = problem["n"]
    return {
        "rp": rp,
        "Rd": Rd,
        "mu": float(np.sum(X * S)) / n,
        "pobj": pobj,
        "dobj": dobj,
        "relgap": abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj)),
        "pinf": float(np.linalg.norm(rp)) / (1.0 + float(np.linalg.norm(b))),
        "dinf": float(np.linalg.norm(Rd)) / (1.0 + float(np.linalg.norm(C))),
    }


def solve(problem, tol=1e-8, maxit=100, step_frac=0.98, newton=None, start=None, verbose=False):
    """Run the IPM.  ``newton`` may replace the direct Newton solve; it is
    called as newton(problem, X, S, G, d, W, bt, Ct, Rd) -> (dX, dy, dS)."""
    n = problem["n"]
    if start is None:
        xi, eta = start_point(problem)
        X = xi * np.eye(n)
        S = eta * np.eye(n)
        y = np.zeros(problem["m"])
    else:
        X, y, S = (np.array(a, dtype=np.float64) for a in start)
    hist = []
    status = "maxit"
    for it in range(maxit + 1):
        res = residuals(problem, X, y, S)
        rec = {k: res[k] for k in ("mu", "pobj", "dobj", "relgap", "pinf", "dinf")}
        hist.append(rec)
        if verbose:
            print(it, rec)
        if res["relgap"] <= tol and res["pinf"] <= tol and res["dinf"] <= tol:
            status = "converged"
            break
        if it == maxit:
            break
        mu, Rd, rp = res["mu"], res["Rd"], res["rp"]
        G, d, L = nt_factor(X, S)
        W = sym(G @ G.T)
        Ginv = np.linalg.inv(G)
        Ls = np.linalg.cholesky(sym(S))

        if newton is None:
            fac = schur_factor(problem, G, W)

            def nsolve(bt, Ct):
                return newton_direct(problem, G, fac, bt, Ct, Rd)

        else:

            def nsolve(bt, Ct):
                return newton(problem, X, S, G, d, W, bt, Ct, Rd)

        # predictor
        dXa, dya, dSa = nsolve(rp, sym(Rd + S))
        ap = min(1.0, max_step(L, dXa))
        ad = min(1.0, max_step(Ls, dSa))
        mu_aff = float(np.sum((X + ap * dXa) * (S + ad * dSa))) / n
        sigma = min(1.0, max(0.0, mu_aff / mu)) ** 3
        # corrector
        Dx = Ginv @ dXa @ Ginv.T
        Ds = G.T @ dSa @ G
        H = -(Dx @ Ds + Ds @ Dx)
        H[np.diag_indices(n)] += 2.0 * (sigma * mu - d * d)
        H = H / (d[:, None] + d[None, :])
        Ct = sym(Rd - Ginv.T @ H @ Ginv)
        dX, dy, dS = nsolve(rp, Ct)
        ap = min(1.0, step_frac * max_step(L, dX))
        ad = min(1.0, step_frac * max_step(Ls, dS))
        X = sym(X + ap * dX)
        y = y + ad * dy
        S = sym(S + ad * dS)
        rec.update({"alpha_p": ap, "alpha_d": ad, "sigma": sigma})
    return {"X": X, "y": y, "S": S, "status": status, "iterations": len(hist) - 1, "history": hist}
