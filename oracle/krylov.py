"""Krylov solvers used on the augmented system.

* ``pcg`` follows Definition pcg: x_{j+1} = x_j + a_j p_j,
  r_{j+1} = r_j - a_j A p_j, P z_{j+1} = r_{j+1}, p_{j+1} = z_{j+1} + b_j p_j,
  a_j = <r_j, z_j> / <p_j, A p_j>.  The printed beta_j = <r_{j+1}, z_j>/<r_j, z_j>
  is read as the standard <r_{j+1}, z_{j+1}>/<r_j, z_j> (with the printed form
  the residuals' P^{-1}-orthogonality makes beta vanish and the method
  degenerates to steepest descent).
* ``solve_newton_pcg`` is Corollary pcg: indefinite PCG on eq. augsys with the
  preconditioner [beta I, A Q; Q^T A^T, -tau^2 Sigma], started from
  [0; -Sigma^{-1} Q^T c], followed by the recovery eq. recover.  P is
  applied through its LU factors (one factorisation per system) with one
  step of iterative refinement, and the residual's bottom block is held at
  zero (Prop. indefpcg): as tau^2 Sigma -> 0 (entries below 1e-17 late in a
  solve) rounding in either would otherwise stall the iteration.
  ``solve_newton_pcg_lp`` is the same with the LP block.
* ``solve_newton_minres`` is Corollary minres: MINRES on eq. augsys with the
  identity preconditioner from 0 (SciPy's MINRES serves as the library step).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import reform as rf


def pcg(apply_a, b, apply_pinv, x0, stop, maxit, keep_x=False, top=None):
    """PCG of Definition pcg.  ``stop(r)`` decides convergence on the residual.

    Returns (x, iterations, residual history); with ``keep_x`` the history
    holds (r_j, x_j) pairs instead of residuals only.  With ``top`` = m the
    residual's entries from m on are held at zero: on eq. augsys started as
    in Corollary pcg they vanish in exact arithmetic (Prop. indefpcg), and
    holding them there keeps rounding in them out of the iteration.
    """
    x = x0.copy()
    r = b - apply_a(x)
    if top is not None:
        r[top:] = 0.0
    z = apply_pinv(r)
    p = z.copy()
    rz = float(r @ z)
    hist = [(r, x.copy()) if keep_x else r]
    it = 0
    while it < maxit and not stop(r):
        Ap = apply_a(p)
        alpha = rz / float(p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        if top is not None:
            r[top:] = 0.0
        z = apply_pinv(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        it += 1
        hist.append((r, x.copy()) if keep_x else r)
    return x, it, hist


def solve_newton_pcg(problem, sp, bt, Ct, beta=None, tol=1e-10, maxit=500):
    """Corollary pcg + eq. recover.  Returns (dX, dy, info)."""
    m = problem["m"]
    E = rf.e_matrix(sp)
    sig = rf.sigma_diag(sp)
    if beta is None:
        beta = rf.beta_rule(sp, problem)
    gu, gv = rf.aug_rhs(problem, sp, E, bt, Ct)
    g = np.concatenate([gu, gv])
    v0 = -rf.qt_apply(sp, Ct) / sig
    x0 = np.concatenate([np.zeros(m), v0])
    AQ = rf.aq_matrix(problem, sp)
    Pm = rf.precond_matrix(AQ, sp, sig, beta)
    P = sla.lu_factor(Pm)

    def apply_k(x):
        t, b_ = rf.aug_apply(problem, sp, E, sig, x[:m], x[m:])
        return np.concatenate([t, b_])

    def apply_pinv(rv):
        # one step of iterative refinement: the bottom equation of P z = r
        # must hold to rounding for the bottom residual to stay zero
        z = sla.lu_solve(P, rv)
        return z + sla.lu_solve(P, rv - Pm @ z)

    r0 = g - apply_k(x0)
    ref = np.linalg.norm(r0[:m])
    ref = ref if ref > 0 else 1.0

    def stop(rv):
        return np.linalg.norm(rv[:m]) <= tol * ref

    x, it, hist = pcg(apply_k, g, apply_pinv, x0, stop, maxit, top=m)
    dX, dy = rf.recover(problem, sp, E, x[:m], x[m:], Ct)
    info = {
        "iterations": it,
        "beta": beta,
        "r": sp["r"],
        "tau": sp["tau"],
        "res_u": [float(np.linalg.norm(h[:m])) for h in hist],
        "res_v": [float(np.linalg.norm(h[m:])) for h in hist],
        "ref": ref,
        "u": x[:m],
        "v": x[m:],
    }
    return dX, dy, info


def solve_newton_pcg_lp(problem, sp, lsp, bt, Ct, ct, beta=None, tol=1e-10, maxit=500):
    """Corollary pcg + eq. recover on the system extended by the LP block.

    Returns (dX, dy, dx, info)."""
    m = problem["m"]
    E = rf.e_matrix(sp)
    sig = rf.sigma_diag(sp)
    sig_all = np.concatenate([sig, lsp["sig"]])
    if beta is None:
        beta = rf.beta_rule_lp(sp, lsp, problem)
    gu, gv = rf.aug_rhs_lp(problem, sp, lsp, E, bt, Ct, ct)
    g = np.concatenate([gu, gv])
    v0 = -np.concatenate([rf.qt_apply(sp, Ct), ct[lsp["T"]]]) / sig_all
    x0 = np.concatenate([np.zeros(m), v0])
    AQ = rf.aq_matrix_lp(problem, sp, lsp)
    Pm = rf.precond_matrix(AQ, sp, sig_all, beta)
    P = sla.lu_factor(Pm)

    def apply_k(x):
        t, b_ = rf.aug_apply_lp(problem, sp, lsp, E, sig, x[:m], x[m:])
        return np.concatenate([t, b_])

    def apply_pinv(rv):
        # one step of iterative refinement: the bottom equation of P z = r
        # must hold to rounding for the bottom residual to stay zero
        z = sla.lu_solve(P, rv)
        return z + sla.lu_solve(P, rv - Pm @ z)

    r0 = g - apply_k(x0)
    ref = np.linalg.norm(r0[:m])
    ref = ref if ref > 0 else 1.0

    def stop(rv):
        return np.linalg.norm(rv[:m]) <= tol * ref

    x, it, hist = pcg(apply_k, g, apply_pinv, x0, stop, maxit, top=m)
    dX, dy, dx = rf.recover_lp(problem, sp, lsp, E, x[:m], x[m:], Ct, ct)
    info = {"iterations": it, "beta": beta, "r": sp["r"], "t": lsp["t"], "tau": sp["tau"], "ref": ref,
            "res_u": [float(np.linalg.norm(h[:m])) for h in hist], "u": x[:m], "v": x[m:]}
    return dX, dy, dx, info


def solve_newton_minres(problem, sp, bt, Ct, tol=1e-10, maxit=5000):
    """Corollary minres + eq. recover.  Returns (dX, dy, info)."""
    from scipy.sparse.linalg import LinearOperator, minres

    m = problem["m"]
    E = rf.e_matrix(sp)
    sig = rf.sigma_diag(sp)
    gu, gv = rf.aug_rhs(problem, sp, E, bt, Ct)
    g = np.concatenate([gu, gv])
    N = g.size

    def apply_k(x):
        t, b_ = rf.aug_apply(problem, sp, E, sig, x[:m], x[m:])
        return np.concatenate([t, b_])

    op = LinearOperator((N, N), matvec=apply_k, dtype=np.float64)
    count = {"it": 0}

    def cb(_):
        count["it"] += 1

    x, flag = minres(op, g, rtol=tol, maxiter=maxit, callback=cb)
    dX, dy = rf.recover(problem, sp, E, x[:m], x[m:], Ct)
    return dX, dy, {"iterations": count["it"], "flag": int(flag), "u": x[:m], "v": x[m:]}
