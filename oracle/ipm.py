"""Plain FP64 primal-dual interior-point method with direct Newton solves.

This is the textbook method the paper accelerates: each Newton subproblem
(Introduction, eq. newt; Section 3, eq. Newt-eps) is solved directly by
forming and factoring the m x m Schur complement M_ij = <A_i, W A_j W>,
which the Introduction names as the standard direct approach.  The outer
loop is an infeasible primal-dual path-following method with the
Nesterov-Todd direction and a Mehrotra predictor-corrector; the paper uses
SeDuMi for this loop and does not spell it out, so both the oracle and the
GPU library follow the same written-out algorithm (coded separately):

1. X = xi I, S = eta I, y = 0 (SDPT3-style magnitudes); an LP block starts
   at x = xi 1, s = eta 1.
2. r_p = b - A(X) - B x, R_d = C - A^T(y) - S, r_d = c - B^T y - s,
   mu = (<X, S> + x^T s) / (n + l); stop when the relative gap, primal and
   dual infeasibility are all <= tol.
3. NT factor G (oracle.nt.nt_factor), W = G G^T, d = diag(G^T S G); for the
   LP block w = sqrt(x / s) and v = sqrt(x s) (the one-dimensional case).
4. Predictor: Newton system with b~ = r_p, C~ = R_d + S, c~ = r_d + s.
5. Step to the boundary of the cones for (X, x) and (S, s) separately;
   sigma = (mu_aff / mu)^3.
6. Corrector: H_ij = [2(sigma mu - d_i^2) delta_ij - (Dx Ds + Ds Dx)_ij]/(d_i+d_j)
   with Dx = G^{-1} dX_a G^{-T}, Ds = G^T dS_a G; C~ = R_d - G^{-T} H G^{-1};
   on the LP block h = (sigma mu - v^2 - dx_a ds_a) / v and c~ = r_d - h / w.
7. Step lengths min(1, 0.98 alpha_max), update, repeat.

In every Newton system dX = W (A^T(dy) - C~) W, dS = R_d - A^T(dy),
dx = w^2 (B^T dy - c~) and ds = r_d - B^T dy, i.e. the KKT system of eq.
Newt-eps with the residual-form dS, extended by the LP block.
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
    if problem["kind"] in ("dense", "sparse"):
        A = (problem["A"].reshape(m, n, n) if problem["kind"] == "dense"
             else np.stack([ops.a_matrix(problem, i) for i in range(m)]))
        At = np.matmul(np.matmul(G.T[None], A), G[None])
    else:
        jk = problem["jk"]
        Gj = G[jk[:, 0]]
        Gk = G[jk[:, 1]]
        At = 0.5 * (Gj[:, :, None] * Gk[:, None, :] + Gk[:, :, None] * Gj[:, None, :])
    return At[:, jj, kk] * w


def schur_matrix(problem, G: np.ndarray, W: np.ndarray, w_lp=None) -> np.ndarray:
    """M_ij = <A_i, W A_j W> (+ (B diag(w_lp^2) B^T)_ij with an LP block) formed explicitly."""
    if problem["kind"] in ("dense", "sparse"):
        Ap = scaled_rows(problem, G)
        M = Ap @ Ap.T
    else:
        jk = problem["jk"]
        j, k = jk[:, 0], jk[:, 1]
        M = 0.5 * (W[np.ix_(j, j)] * W[np.ix_(k, k)] + W[np.ix_(j, k)] * W[np.ix_(k, j)])
    if w_lp is not None:
        B = ops.b_matrix(problem)
        M = M + (B * (w_lp * w_lp)) @ B.T
    return M


def schur_factor(problem, G: np.ndarray, W: np.ndarray, w_lp=None):
    """Thin QR of A~^T (rows [svec(G^T A_i G), (B diag(w_lp))_i]): A~^T = Q1 R, so M = R^T R.

    Factoring A~ instead of M avoids squaring the condition number; M itself
    becomes too ill-conditioned for a Cholesky factorisation as mu -> 0,
    which is the difficulty the Introduction attributes to the direct
    approach.
    """
    Ap = scaled_rows(problem, G)
    if w_lp is not None:
        Ap = np.hstack([Ap, ops.b_matrix(problem) * w_lp])
    Q1, R = np.linalg.qr(Ap.T, mode="reduced")
    return Ap, Q1, R


def newton_direct(problem, G, fac, bt, Ct, Rd, lp=None):
    """Direct solve of eq. Newt-eps in NT-scaled coordinates.

    With dX = G Z G^T (and dx = w z_lp on an LP block) the Newton subproblem
    (eq. newt) becomes min 1/2 ||z||^2 + cbar^T z  s.t.  A~ z = b~, where
    z = [svec(Z); z_lp] and cbar = [svec(G^T C~ G); w c~]; its KKT conditions
    are z = A~^T dy - cbar and A~ A~^T dy = b~ + A~ cbar, i.e.
    M dy = b~ + A(W C~ W) + B diag(w^2) c~ with dX = W (A^T(dy) - C~) W.
    With A~^T = Q1 R: w = R^{-T}(b~ + A~ cbar), A~^T dy = Q1 w and dy = R^{-1} w.
    ``lp`` = (w, c~, r_d) for a problem with an LP block; the return value is
    then (dX, dy, dS, dx, ds).
    """
    Ap, Q1, R = fac
    n = problem["n"]
    jj, kk = np.tril_indices(n)
    wts = np.where(jj == kk, 1.0, np.sqrt(2.0))
    GCG = G.T @ Ct @ G
    cbar = GCG[jj, kk] * wts
    if lp is not None:
        w_lp, ct_lp, rd_lp = lp
        cbar = np.concatenate([cbar, w_lp * ct_lp])
    w = sla.solve_triangular(R, bt + Ap @ cbar, trans="T")
    dy = sla.solve_triangular(R, w)
    z = Q1 @ w - cbar
    nz = jj.size
    Z = np.zeros((n, n))
    Z[jj, kk] = z[:nz] / wts
    Z[kk, jj] = z[:nz] / wts
    dX = sym(G @ Z @ G.T)
    dS = sym(Rd - ops.at_op(problem, dy))
    if lp is None:
        return dX, dy, dS
    dx = w_lp * z[nz:]
    ds = rd_lp - ops.bt_op(problem, dy)
    return dX, dy, dS, dx, ds


def max_step(L: np.ndarray, D: np.ndarray) -> float:
    """Largest alpha with L L^T + alpha D PSD: 1 / max(0, -lambda_min(L^{-1} D L^{-T}))."""
    T = sla.solve_triangular(L, D, lower=True)
    T = sla.solve_triangular(L, T.T, lower=True)
    lmin = float(np.linalg.eigvalsh(sym(T))[0])
    return np.inf if lmin >= 0 else -1.0 / lmin


def max_step_lp(x: np.ndarray, dx: np.ndarray) -> float:
    """Largest alpha with x + alpha dx >= 0 (ratio test)."""
    neg = dx < 0
    return np.inf if not np.any(neg) else float(np.min(-x[neg] / dx[neg]))


def residuals(problem, X, y, S, x=None, s=None):
    b, C = problem["b"], problem["C"]
    rp = b - ops.a_op(problem, X)
    Rd = sym(C - ops.at_op(problem, y) - S)
    pobj = float(np.sum(C * X))
    dobj = float(b @ y)
    n = problem["n"]
    gap = float(np.sum(X * S))
    dnorm2, cnorm2 = float(np.sum(Rd * Rd)), float(np.sum(C * C))
    out = {}
    if ops.has_lp(problem):
        c = problem["lp"]["c"]
        rp = rp - ops.b_op(problem, x)
        rd = c - ops.bt_op(problem, y) - s
        pobj += float(c @ x)
        gap += float(x @ s)
        n += c.size
        dnorm2 += float(rd @ rd)
        cnorm2 += float(c @ c)
        out["rd"] = rd
    out.update({
        "rp": rp,
        "Rd": Rd,
        "mu": gap / n,
        "pobj": pobj,
        "dobj": dobj,
        "relgap": abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj)),
        "pinf": float(np.linalg.norm(rp)) / (1.0 + float(np.linalg.norm(b))),
        "dinf": float(np.sqrt(dnorm2)) / (1.0 + float(np.sqrt(cnorm2))),
    })
    return out


def solve(problem, tol=1e-8, maxit=100, step_frac=0.98, newton=None, start=None, verbose=False):
    """Run the IPM.  ``newton`` may replace the direct Newton solve; it is
    called as newton(problem, X, S, G, d, W, bt, Ct, Rd) -> (dX, dy, dS), and
    for a problem with an LP block with the extra keyword
    lp=(x, s, w, c~, r_d) -> (dX, dy, dS, dx, ds)."""
    n = problem["n"]
    with_lp = ops.has_lp(problem)
    ell = ops.lp_len(problem)
    if start is None:
        xi, eta = start_point(problem)
        X = xi * np.eye(n)
        S = eta * np.eye(n)
        y = np.zeros(problem["m"])
        x = np.full(ell, xi)
        s = np.full(ell, eta)
    else:
        X, y, S = (np.array(a, dtype=np.float64) for a in start[:3])
        x, s = ((np.array(a, dtype=np.float64) for a in start[3:5]) if with_lp else (np.zeros(0), np.zeros(0)))
    hist = []
    status = "maxit"
    for it in range(maxit + 1):
        res = residuals(problem, X, y, S, x, s)
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
        rd = res.get("rd")
        G, d, L = nt_factor(X, S)
        W = sym(G @ G.T)
        Ginv = np.linalg.inv(G)
        Ls = np.linalg.cholesky(sym(S))
        w_lp = np.sqrt(x / s) if with_lp else None
        v_lp = np.sqrt(x * s) if with_lp else None

        if newton is None:
            fac = schur_factor(problem, G, W, w_lp)

            def nsolve(bt, Ct, ct=None):
                return newton_direct(problem, G, fac, bt, Ct, Rd, (w_lp, ct, rd) if with_lp else None)

        else:

            def nsolve(bt, Ct, ct=None):
                if with_lp:
                    return newton(problem, X, S, G, d, W, bt, Ct, Rd, lp=(x, s, w_lp, ct, rd))
                return newton(problem, X, S, G, d, W, bt, Ct, Rd)

        def steps(dX, dS, dx, ds, frac):
            ap = min(1.0, frac * max_step(L, dX))
            ad = min(1.0, frac * max_step(Ls, dS))
            if with_lp:
                ap = min(ap, frac * max_step_lp(x, dx))
                ad = min(ad, frac * max_step_lp(s, ds))
            return ap, ad

        # predictor
        out = nsolve(rp, sym(Rd + S), (rd + s) if with_lp else None)
        dXa, dya, dSa = out[:3]
        dxa, dsa = out[3:] if with_lp else (np.zeros(0), np.zeros(0))
        ap, ad = steps(dXa, dSa, dxa, dsa, 1.0)
        gap_aff = float(np.sum((X + ap * dXa) * (S + ad * dSa))) + float((x + ap * dxa) @ (s + ad * dsa))
        mu_aff = gap_aff / (n + ell)
        sigma = min(1.0, max(0.0, mu_aff / mu)) ** 3
        # corrector
        Dx = Ginv @ dXa @ Ginv.T
        Ds = G.T @ dSa @ G
        H = -(Dx @ Ds + Ds @ Dx)
        H[np.diag_indices(n)] += 2.0 * (sigma * mu - d * d)
        H = H / (d[:, None] + d[None, :])
        Ct = sym(Rd - Ginv.T @ H @ Ginv)
        ct = None
        if with_lp:
            h = (sigma * mu - v_lp * v_lp - dxa * dsa) / v_lp
            ct = rd - h / w_lp
        out = nsolve(rp, Ct, ct)
        dX, dy, dS = out[:3]
        dx, ds = out[3:] if with_lp else (np.zeros(0), np.zeros(0))
        ap, ad = steps(dX, dS, dx, ds, step_frac)
        X = sym(X + ap * dX)
        y = y + ad * dy
        S = sym(S + ad * dS)
        x = x + ap * dx
        s = s + ad * ds
        rec.update({"alpha_p": ap, "alpha_d": ad, "sigma": sigma})
    out = {"X": X, "y": y, "S": S, "status": status, "iterations": len(hist) - 1, "history": hist}
    if with_lp:
        out.update({"x": x, "s": s})
    return out
