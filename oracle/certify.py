"""KKT certificate of a primal-dual point (problem statement, eq. sdp-pd).

For any returned (X, y, S) this measures, in FP64 on the CPU:
primal infeasibility ||b - A(X)|| / (1 + ||b||), dual infeasibility
||C - A^T(y) - S||_F / (1 + ||C||_F), the relative duality gap
|<C,X> - b^T y| / (1 + |<C,X>| + |b^T y|), the smallest eigenvalues of X
and S, mu = <X,S>/n and the centrality ||X^{1/2} S X^{1/2} / mu - I||
(the quantity bounded by delta in Assumption 1).

With an LP block (x, s >= 0; A(X) + B x = b, B^T y + s = c, cost c^T x as
in eq. rmc-sdp) the residuals, objective and mu include it, and the
smallest entries of x and s are reported beside the eigenvalues.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from .notation import sym


def certificate(problem, X, y, S, x=None, s=None):
    n = problem["n"]
    b, C = problem["b"], problem["C"]
    X = sym(np.asarray(X, dtype=np.float64))
    S = sym(np.asarray(S, dtype=np.float64))
    y = np.asarray(y, dtype=np.float64)
    rp = b - ops.a_op(problem, X)
    Rd = C - ops.at_op(problem, y) - S
    pobj = float(np.sum(C * X))
    dobj = float(b @ y)
    dn2, cn2 = float(np.sum(Rd * Rd)), float(np.sum(C * C))
    wx, Vx = np.linalg.eigh(X)
    ws = np.linalg.eigvalsh(S)
    gap, cnt = float(np.sum(X * S)), n
    out = {}
    if ops.has_lp(problem):
        c = problem["lp"]["c"]
        x = np.asarray(x, dtype=np.float64)
        s = np.asarray(s, dtype=np.float64)
        rp = rp - ops.b_op(problem, x)
        rd = c - ops.bt_op(problem, y) - s
        pobj += float(c @ x)
        dn2 += float(rd @ rd)
        cn2 += float(c @ c)
        gap += float(x @ s)
        cnt += c.size
        out.update({"min_x": float(x.min()), "min_s": float(s.min())})
    mu = gap / cnt
    Xh = (Vx * np.sqrt(np.clip(wx, 0.0, None))) @ Vx.T
    mu_sdp = float(np.sum(X * S)) / n
    if mu_sdp > 0:
        # spectral norm of a symmetric matrix = its largest eigenvalue in magnitude
        delta = float(np.abs(np.linalg.eigvalsh(sym(Xh @ S @ Xh / mu_sdp - np.eye(n)))).max())
    else:
        delta = float("inf")
    out.update({
        "pinf": float(np.linalg.norm(rp)) / (1.0 + float(np.linalg.norm(b))),
        "dinf": float(np.sqrt(dn2)) / (1.0 + float(np.sqrt(cn2))),
        "relgap": abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj)),
        "pobj": pobj,
        "dobj": dobj,
        "lmin_X": float(wx[0]),
        "lmin_S": float(ws[0]),
        "mu": mu,
        "delta": delta,
    })
    return out
