"""Low-rank plus well-conditioned reformulation of the Newton system.

Follows Section 3 of the paper:

* eq. EQSigdef: split W = Q Lam Q^T + Qp Lamp Qp^T (top r eigenvalues and the
  rest), tau = lambda_{r+1}(W)/2,
  script-E = E (x)_s E with E = Q Q^T + Qp Lamp Qp^T / tau,
  script-Q = [Q (x)_s Q, sqrt(2) Psi_n^T (Q (x) Qp)],
  Sigma = diag(Lam (x)_s Lam - tau^2 I, (Lam - tau I) (x) Lamp)^{-1}.
* eq. augsys / eq. recover (together eq. augrec): the augmented system
  [A E A^T, A Q; Q^T A^T, -tau^2 Sigma][u; v] = [b + tau^2 A E c; tau^2 Q^T c]
  and the recovery dy = u / tau^2, svec(dX) = E(A^T u - tau^2 c) + Q v.
* Section 5: matrix-free products E svec(X) = svec(E X E),
  Q [svec(B); vec(N)] = svec([Q Qp][B; sqrt(2) N] Q^T),
  Q^T svec(X) = [svec(Q^T X Q); sqrt(2) vec(Qp^T X Q)].
* Section 6 / Corollary pcg: the indefinite preconditioner
  [beta I, A Q; Q^T A^T, -tau^2 Sigma] and its Schur complement
  C = tau^2 Sigma + A Q^T A Q / beta.
* Experiments section: rank rule r = argmax_{i <= rhat} lambda_i / lambda_{i+1}
  and beta = (median eigenvalue of E)^2.

LP block (eq. rmc-sdp, eq. snl-sdp; the paper gives no formulas for it):
each coordinate x_j >= 0 is a 1 x 1 block of the cone with scaling
w_j = sqrt(x_j / s_j), so the Schur complement gains B diag(w^2) B^T.  The
split treats w_j like an eigenvalue of W: the coordinates with w_j > 2 tau
(above lambda_{r+1}) join the low-rank part, T = those indices (at most
``cap`` of them: j stays only when at most cap entries are >= w_j), with
script-E entry 1 and Sigma entry
1/(w_j^2 - tau^2); the others stay in script-E with entry (w_j/tau)^2 <= 4.
Then diag(w^2) = tau^2 script-E_lp + P_T Sigma_lp^{-1} P_T^T exactly, the
LP analogue of W (x)_s W = tau^2 script-E + script-Q Sigma^{-1} script-Q^T,
and the augmented system, right-hand side, recovery and preconditioner
extend block by block: v = [v_sdp; v_lp], script-A script-Q gains the
columns B[:, T], and dx = script-E_lp (B^T u - tau^2 c~) + P_T v_lp.

Readings (documented in the design notes):
* the v-coordinates are [svec(B) (r(r+1)/2); vec(N) ((n-r) x r, column-major)];
* eigenvalues are sorted in decreasing order and every eigenvector column is
  signed so that its entry of largest magnitude (lowest index on ties) is
  positive, which fixes the basis whenever the eigenvalues are distinct;
* on a tie in the rank rule the smallest i is taken;
* beta is the squared median eigenvalue of E multiplied by the mean of
  ||A_i||_F^2, so that it stays inside [lambda_min, lambda_max] of
  A E A^T for constraint matrices that are not unit-norm; the median of an
  even count is the mean of the two middle values.  With the LP block it is
  raised to the largest diagonal entry of B diag(e2) B^T when that is
  larger (beta_rule_lp).
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from .notation import SQRT2, psi, skron, smat, svec, sym


def canonical_signs(V: np.ndarray) -> np.ndarray:
    idx = np.argmax(np.abs(V), axis=0)
    s = np.sign(V[idx, np.arange(V.shape[1])])
    s[s == 0] = 1.0
    return V * s


def eig_split(W: np.ndarray, rank_max: int = 10, rank_fixed: int = 0):
    """Eigen-split of the scaling point per eq. EQSigdef and the rank rule."""
    lam, V = np.linalg.eigh(sym(W))
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    V = canonical_signs(V[:, order])
    n = lam.size
    if rank_fixed > 0:
        r = min(rank_fixed, n - 1)
    else:
        rhat = max(1, min(rank_max, n - 1))
        ratios = lam[:rhat] / lam[1 : rhat + 1]
        r = int(np.argmax(ratios)) + 1
    tau = 0.5 * lam[r]
    return {
        "n": n,
        "r": r,
        "tau": tau,
        "lam": lam,
        "V": V,
        "Q": V[:, :r],
        "Qp": V[:, r:],
        "lam_top": lam[:r],
        "lam_perp": lam[r:],
    }


def dim_d(n: int, r: int) -> int:
    return n * r - r * (r - 1) // 2


def e_matrix(sp) -> np.ndarray:
    """E = Q Q^T + tau^{-1} Qp Lamp Qp^T."""
    Q, Qp = sp["Q"], sp["Qp"]
    return Q @ Q.T + (Qp * (sp["lam_perp"] / sp["tau"])) @ Qp.T


def e_eigenvalues(sp) -> np.ndarray:
    return np.concatenate([np.ones(sp["r"]), sp["lam_perp"] / sp["tau"]])


def sigma_diag(sp) -> np.ndarray:
    """Diagonal of Sigma in v-coordinate order."""
    r, n, tau = sp["r"], sp["n"], sp["tau"]
    lt, lp = sp["lam_top"], sp["lam_perp"]
    sb = []
    for j in range(r):
        for i in range(j, r):
            sb.append(1.0 / (lt[i] * lt[j] - tau * tau))
    sn = np.empty((n - r, r))
    for j in range(r):
        sn[:, j] = 1.0 / ((lt[j] - tau) * lp)
    return np.concatenate([np.array(sb), sn.reshape(-1, order="F")])


def beta_rule(sp, problem) -> float:
    med = float(np.median(e_eigenvalues(sp)))
    scale = float(np.mean(ops.frob_norms(problem) ** 2))
    return med * med * scale


def beta_rule_lp(sp, lsp, problem) -> float:
    """beta with the LP block: the (1,1) block of eq. augsys becomes
    A E A^T + B diag(e2) B^T, and beta is the SDP rule's value raised to the
    largest diagonal entry of B diag(e2) B^T when that is larger.  A diagonal
    entry of that positive semidefinite term is at most lambda_max of the
    whole block, so beta stays inside the bracket of Corollary pcg."""
    B = ops.b_matrix(problem)
    diag = (B * B) @ lsp["e2"]
    return max(beta_rule(sp, problem), float(diag.max()) if diag.size else 0.0)


# ---- explicit matrices (small n only) ---------------------------------------


def e_bold(sp) -> np.ndarray:
    E = e_matrix(sp)
    return skron(E, E)


def q_bold(sp) -> np.ndarray:
    Q, Qp = sp["Q"], sp["Qp"]
    n = sp["n"]
    QB = skron(Q, Q)
    QN = SQRT2 * psi(n).T @ np.kron(Q, Qp)
    return np.hstack([QB, QN])


def ws_kron(W: np.ndarray) -> np.ndarray:
    """W (x)_s W from the definition of the symmetric Kronecker product."""
    return skron(W, W)


# ---- matrix-free products (Section 5) ---------------------------------------


def q_apply(sp, v: np.ndarray) -> np.ndarray:
    """Matrix whose svec is script-Q v: sym([Q Qp][B; sqrt(2) N] Q^T)."""
    n, r = sp["n"], sp["r"]
    nb = r * (r + 1) // 2
    B = smat(v[:nb], r)
    N = v[nb:].reshape((n - r, r), order="F")
    U = sp["Q"] @ B + SQRT2 * sp["Qp"] @ N
    return sym(U @ sp["Q"].T)


def qt_apply(sp, X: np.ndarray) -> np.ndarray:
    """script-Q^T svec(X) = [svec(Q^T X Q); sqrt(2) vec(Qp^T X Q)]."""
    XQ = sym(X) @ sp["Q"]
    top = sp["Q"].T @ XQ
    bot = sp["Qp"].T @ XQ
    return np.concatenate([svec(top), SQRT2 * bot.reshape(-1, order="F")])


def aug_apply(problem, sp, E, sig, u, v):
    """[A E A^T, A Q; Q^T A^T, -tau^2 Sigma] [u; v] by the Section 5 formulas."""
    Y = ops.at_op(problem, u)
    top = ops.a_op(problem, E @ Y @ E + q_apply(sp, v))
    bot = qt_apply(sp, Y) - sp["tau"] ** 2 * sig * v
    return top, bot


def aug_rhs(problem, sp, E, bt, Ct):
    """[b + tau^2 A E c; tau^2 Q^T c] (eq. augsys)."""
    t2 = sp["tau"] ** 2
    return bt + t2 * ops.a_op(problem, E @ Ct @ E), t2 * qt_apply(sp, Ct)


def recover(problem, sp, E, u, v, Ct):
    """dy = u / tau^2, dX = E(A^T u - tau^2 C) E + Q v (eq. recover)."""
    t2 = sp["tau"] ** 2
    dy = u / t2
    dX = E @ (ops.at_op(problem, u) - t2 * Ct) @ E + q_apply(sp, v)
    return sym(dX), dy


def aq_matrix(problem, sp) -> np.ndarray:
    """script-A script-Q, row i = (script-Q^T svec(A_i))^T."""
    m = problem["m"]
    out = np.empty((m, dim_d(sp["n"], sp["r"])))
    for i in range(m):
        out[i] = qt_apply(sp, ops.a_matrix(problem, i))
    return out


def aug_matrix(problem, sp) -> np.ndarray:
    """The augmented matrix of eq. augsys assembled from explicit blocks."""
    Am = ops.amat(problem)
    Eb = e_bold(sp)
    Qb = q_bold(sp)
    sig = sigma_diag(sp)
    AQ = Am @ Qb
    top = np.hstack([Am @ Eb @ Am.T, AQ])
    bot = np.hstack([AQ.T, -(sp["tau"] ** 2) * np.diag(sig)])
    return np.vstack([top, bot])


def precond_matrix(AQ: np.ndarray, sp, sig: np.ndarray, beta: float) -> np.ndarray:
    """[beta I, A Q; Q^T A^T, -tau^2 Sigma] (Corollary pcg)."""
    m = AQ.shape[0]
    top = np.hstack([beta * np.eye(m), AQ])
    bot = np.hstack([AQ.T, -(sp["tau"] ** 2) * np.diag(sig)])
    return np.vstack([top, bot])


def schur_c(AQ: np.ndarray, sp, sig: np.ndarray, beta: float) -> np.ndarray:
    """C = tau^2 Sigma + beta^{-1} (A Q)^T (A Q) (Section 6)."""
    return (sp["tau"] ** 2) * np.diag(sig) + (AQ.T @ AQ) / beta


# ---- LP block (nonnegative orthant) ------------------------------------------


def lp_split(sp, w: np.ndarray, cap: int | None = None):
    """Split of the LP scaling w = sqrt(x/s) against the SDP split's tau."""
    tau = sp["tau"]
    T = np.flatnonzero(w > 2.0 * tau)
    if cap is not None and T.size > cap:
        # keep j when at most cap entries are >= w_j (a tied group that would
        # overflow the cap stays out as a whole)
        ws = np.sort(w)
        at_least = w.size - np.searchsorted(ws, w[T], side="left")
        T = T[at_least <= cap]
    e2 = (w / tau) ** 2
    e2[T] = 1.0
    sig = 1.0 / (w[T] ** 2 - tau * tau)
    return {"T": T, "e2": e2, "sig": sig, "w": w, "t": int(T.size)}


def aug_apply_lp(problem, sp, lsp, E, sig, u, v):
    """eq. augsys with the LP block: v = [v_sdp; v_lp]."""
    d = sig.size
    top, bot = aug_apply(problem, sp, E, sig, u, v[:d])
    B = ops.b_matrix(problem)
    T = lsp["T"]
    t = B.T @ u
    top = top + B @ (lsp["e2"] * t) + B[:, T] @ v[d:]
    bot_lp = t[T] - sp["tau"] ** 2 * lsp["sig"] * v[d:]
    return top, np.concatenate([bot, bot_lp])


def aug_rhs_lp(problem, sp, lsp, E, bt, Ct, ct):
    t2 = sp["tau"] ** 2
    gu, gv = aug_rhs(problem, sp, E, bt, Ct)
    B = ops.b_matrix(problem)
    gu = gu + t2 * (B @ (lsp["e2"] * ct))
    return gu, np.concatenate([gv, t2 * ct[lsp["T"]]])


def recover_lp(problem, sp, lsp, E, u, v, Ct, ct):
    """eq. recover with the LP block: returns (dX, dy, dx)."""
    d = v.size - lsp["t"]
    dX, dy = recover(problem, sp, E, u, v[:d], Ct)
    t2 = sp["tau"] ** 2
    dx = lsp["e2"] * (ops.bt_op(problem, u) - t2 * ct)
    dx[lsp["T"]] += v[d:]
    return dX, dy, dx


def aq_matrix_lp(problem, sp, lsp) -> np.ndarray:
    """[script-A script-Q, B[:, T]]."""
    return np.hstack([aq_matrix(problem, sp), ops.b_matrix(problem)[:, lsp["T"]]])


def aug_matrix_lp(problem, sp, lsp) -> np.ndarray:
    """The augmented matrix with the LP block, from explicit blocks."""
    Am = ops.amat(problem)
    B = ops.b_matrix(problem)
    AQ = np.hstack([Am @ q_bold(sp), B[:, lsp["T"]]])
    sig = np.concatenate([sigma_diag(sp), lsp["sig"]])
    top = np.hstack([Am @ e_bold(sp) @ Am.T + (B * lsp["e2"]) @ B.T, AQ])
    bot = np.hstack([AQ.T, -(sp["tau"] ** 2) * np.diag(sig)])
    return np.vstack([top, bot])
