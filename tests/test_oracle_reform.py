"""Pins for the oracle's reformulation (Sections 3, 5 and 6) and Krylov solvers."""
import numpy as np
import pytest

import workloads
from oracle import ipm, krylov, nt, operators as ops, reform as rf
from oracle.notation import smat, svec, sym


def split_w(n, r, seed, ratio=1e3):
    """A PD W whose top r eigenvalues sit `ratio` above the rest."""
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    top = np.sqrt(ratio) * rng.uniform(1.0, 3.0, size=r)
    bot = rng.uniform(0.2, 1.0, size=n - r) / np.sqrt(ratio)
    w = np.concatenate([np.sort(top)[::-1], np.sort(bot)[::-1]])
    return (Qm * w) @ Qm.T, w


@pytest.mark.parametrize("r", [1, 2, 3])
def test_prop_correct_identity(r):
    # Proposition correct / Appendix A: W (x)_s W = Q Sigma^{-1} Q^T + tau^2 E.
    W, _ = split_w(6, r, seed=r)
    sp = rf.eig_split(W, rank_fixed=r)
    Qb = rf.q_bold(sp)
    sig = rf.sigma_diag(sp)
    lhs = rf.ws_kron(W)
    rhs = Qb @ np.diag(1.0 / sig) @ Qb.T + sp["tau"] ** 2 * rf.e_bold(sp)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(lhs).max())
    assert np.all(sig > 0)
    assert np.linalg.eigvalsh(rf.e_bold(sp))[0] > 0


@pytest.mark.parametrize("n,r", [(5, 1), (6, 2), (7, 3)])
def test_lemma_spanq(n, r):
    # Lemma spanQ: Q^T Q = I_d with d = nr - r(r-1)/2, colspan Q = {svec(V Q^T)}.
    W, _ = split_w(n, r, seed=10 + n)
    sp = rf.eig_split(W, rank_fixed=r)
    Qb = rf.q_bold(sp)
    d = rf.dim_d(n, r)
    assert Qb.shape == (n * (n + 1) // 2, d)
    assert np.allclose(Qb.T @ Qb, np.eye(d), atol=1e-13)
    rng = np.random.default_rng(0)
    for _ in range(3):
        V = rng.standard_normal((n, r))
        s = svec(V @ sp["Q"].T)
        proj = Qb @ (Qb.T @ s)
        assert np.allclose(proj, s, atol=1e-12)


@pytest.mark.parametrize("r", [1, 2])
def test_lemma_eigen_bounds(r):
    # Lemma eigen: 4 >= lmax(E) >= lmin(E) >= w_n^2/w_{r+1}^2 and
    # w_{r+1}^2/(w_n w_r) >= tau^2 lmax(Sigma) >= tau^2 lmin(Sigma) >= w_n^2/(4 w_1^2).
    W, w = split_w(6, r, seed=20 + r, ratio=10.0)
    sp = rf.eig_split(W, rank_fixed=r)
    ev = np.linalg.eigvalsh(rf.e_bold(sp))
    t2s = sp["tau"] ** 2 * rf.sigma_diag(sp)
    lam = sp["lam"]
    assert 4.0 + 1e-12 >= ev[-1] >= ev[0] >= lam[-1] ** 2 / lam[r] ** 2 - 1e-12
    assert lam[r] ** 2 / (lam[-1] * lam[r - 1]) + 1e-12 >= t2s.max() >= t2s.min() >= lam[-1] ** 2 / (4 * lam[0] ** 2) - 1e-15


def test_section5_matvec_formulas():
    # Section 5: E svec(X) = svec(EXE); Q [svec B; vec N] = svec([Q Qp][B; sqrt2 N] Q^T);
    # Q^T svec(X) = [svec(Q^T X Q); sqrt2 vec(Qp^T X Q)], against the explicit Kronecker forms.
    rng = np.random.default_rng(4)
    n, r = 6, 2
    W, _ = split_w(n, r, seed=4)
    sp = rf.eig_split(W, rank_fixed=r)
    E = rf.e_matrix(sp)
    X = sym(rng.standard_normal((n, n)))
    v = rng.standard_normal(rf.dim_d(n, r))
    assert np.allclose(rf.e_bold(sp) @ svec(X), svec(E @ X @ E), atol=1e-12)
    assert np.allclose(rf.q_bold(sp) @ v, svec(rf.q_apply(sp, v)), atol=1e-12)
    assert np.allclose(rf.q_bold(sp).T @ svec(X), rf.qt_apply(sp, X), atol=1e-12)


def small_problem(kind="dense", seed=0):
    if kind == "dense":
        return workloads.gaussian_sensing(7, 2, 18, seed=seed)
    return workloads.matrix_completion(7, 2, 18, seed=seed)


def ipm_point(p, iters):
    """An iterate of the oracle IPM after `iters` iterations."""
    res = ipm.solve(p, maxit=iters)
    return res["X"], res["y"], res["S"]


@pytest.mark.parametrize("kind", ["dense", "entry"])
def test_aug_apply_matches_explicit(kind):
    p = small_problem(kind)
    X, y, S = ipm_point(p, 4)
    G, d, L = nt.nt_factor(X, S)
    sp = rf.eig_split(G @ G.T, rank_max=3)
    rng = np.random.default_rng(5)
    K = rf.aug_matrix(p, sp)
    x = rng.standard_normal(K.shape[0])
    t, b = rf.aug_apply(p, sp, rf.e_matrix(sp), rf.sigma_diag(sp), x[: p["m"]], x[p["m"] :])
    ref = K @ x
    assert np.allclose(np.concatenate([t, b]), ref, atol=1e-11 * np.abs(ref).max())
    assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())


@pytest.mark.parametrize("kind", ["dense", "entry"])
@pytest.mark.parametrize("iters", [2, 6])
def test_augrec_equals_direct_newton(kind, iters):
    # eq. augrec: solving eq. augsys exactly and recovering gives the eq. Newt-eps solution.
    p = small_problem(kind, seed=3)
    X, y, S = ipm_point(p, iters)
    G, d, L = nt.nt_factor(X, S)
    W = sym(G @ G.T)
    sp = rf.eig_split(W, rank_max=3)
    res = ipm.residuals(p, X, y, S)
    Ct = sym(res["Rd"] + S)
    bt = res["rp"]
    fac = ipm.schur_factor(p, G, W)
    dX0, dy0, _ = ipm.newton_direct(p, G, fac, bt, Ct, res["Rd"])
    E = rf.e_matrix(sp)
    gu, gv = rf.aug_rhs(p, sp, E, bt, Ct)
    sol = np.linalg.solve(rf.aug_matrix(p, sp), np.concatenate([gu, gv]))
    dX, dy = rf.recover(p, sp, E, sol[: p["m"]], sol[p["m"] :], Ct)
    assert np.allclose(dX, dX0, rtol=1e-7, atol=1e-8 * np.abs(dX0).max())
    assert np.allclose(dy, dy0, rtol=1e-7, atol=1e-8 * np.abs(dy0).max())


def test_direct_newton_solves_unsubstituted_system():
    # The KKT system of eq. Newt-eps in its original form: A(dX) = b~,
    # A^T(dy) + dS = R_d and dX + W dS W = W (R_d - C~) W.
    p = small_problem("dense", seed=7)
    X, y, S = ipm_point(p, 3)
    G, d, L = nt.nt_factor(X, S)
    W = sym(G @ G.T)
    res = ipm.residuals(p, X, y, S)
    rng = np.random.default_rng(1)
    Ct = sym(rng.standard_normal((7, 7)))
    bt = rng.standard_normal(p["m"])
    dX, dy, dS = ipm.newton_direct(p, G, ipm.schur_factor(p, G, W), bt, Ct, res["Rd"])
    assert np.allclose(ops.a_op(p, dX), bt, atol=1e-10 * np.abs(bt).max())
    assert np.allclose(ops.at_op(p, dy) + dS, res["Rd"], atol=1e-12)
    lhs = dX + W @ dS @ W
    rhs = W @ (res["Rd"] - Ct) @ W
    assert np.allclose(lhs, rhs, atol=1e-9 * np.abs(rhs).max())
    # M = R^T R with M_ij = <A_i, W A_j W>
    _, _, R = ipm.schur_factor(p, G, W)
    M = np.array([[np.sum(ops.a_matrix(p, i) * (W @ ops.a_matrix(p, j) @ W)) for j in range(p["m"])] for i in range(p["m"])])
    assert np.allclose(R.T @ R, M, rtol=1e-10, atol=1e-12 * np.abs(M).max())


@pytest.mark.parametrize("kind", ["dense", "entry"])
def test_schur_matrix_matches_definition(kind):
    # M_ij = <A_i, W A_j W> written out with the explicit matrices A_i, against
    # the oracle's two ways of forming it: the closed form for entry sampling
    # (M_(jk),(pq) = (W_jp W_kq + W_jq W_kp) / 2) or A~ A~^T for dense rows,
    # and R^T R from the thin QR of the scaled rows.  The entry instance has
    # diagonal and off-diagonal pairs, so both halves of the closed form count.
    p = small_problem(kind, seed=3)
    X, y, S = ipm_point(p, 2)
    G, d, L = nt.nt_factor(X, S)
    W = sym(G @ G.T)
    if kind == "entry":
        jk = p["jk"]
        assert np.any(jk[:, 0] == jk[:, 1]) and np.any(jk[:, 0] != jk[:, 1])
    m = p["m"]
    A = [ops.a_matrix(p, i) for i in range(m)]
    M = np.array([[np.sum(A[i] * (W @ A[j] @ W)) for j in range(m)] for i in range(m)])
    got = ipm.schur_matrix(p, G, W)
    assert np.allclose(got, M, rtol=1e-12, atol=1e-13 * np.abs(M).max())
    _, _, R = ipm.schur_factor(p, G, W)
    assert np.allclose(R.T @ R, M, rtol=1e-10, atol=1e-12 * np.abs(M).max())


def test_lemma_smallres():
    # Lemma smallres: with residual [p; d] of eq. augsys, the recovered (x, y)
    # has eq. Newt-eps residual [tau^-2 E^-1 Q C^-1 d; p], C = tau^2 Sigma + Q^T E^-1 Q.
    p = small_problem("dense", seed=11)
    X, y, S = ipm_point(p, 3)
    G, d, L = nt.nt_factor(X, S)
    W = sym(G @ G.T)
    sp = rf.eig_split(W, rank_max=3)
    m = p["m"]
    rng = np.random.default_rng(2)
    Ct = sym(rng.standard_normal((7, 7)))
    bt = rng.standard_normal(m)
    E = rf.e_matrix(sp)
    gu, gv = rf.aug_rhs(p, sp, E, bt, Ct)
    u = rng.standard_normal(m)
    v = rng.standard_normal(rf.dim_d(7, sp["r"]))
    K = rf.aug_matrix(p, sp)
    res = K @ np.concatenate([u, v]) - np.concatenate([gu, gv])
    pr, dr = res[:m], res[m:]
    dX, dy = rf.recover(p, sp, E, u, v, Ct)
    Am = ops.amat(p)
    Db = rf.ws_kron(W)
    c = svec(Ct)
    top = -np.linalg.solve(Db, svec(dX)) + Am.T @ dy - c
    bot = Am @ svec(dX) - bt
    Eb = rf.e_bold(sp)
    Qb = rf.q_bold(sp)
    Cl = sp["tau"] ** 2 * np.diag(rf.sigma_diag(sp)) + Qb.T @ np.linalg.solve(Eb, Qb)
    pred_top = np.linalg.solve(Eb, Qb @ np.linalg.solve(Cl, dr)) / sp["tau"] ** 2
    assert np.allclose(bot, pr, atol=1e-9 * np.abs(pr).max())
    assert np.allclose(top, pred_top, rtol=1e-6, atol=1e-7 * np.abs(pred_top).max())


def test_prop_indefpcg_iterates():
    # Proposition indefpcg: PCG on [A B; B^T -C] with preconditioner [P B; B^T -C]
    # started at [x0; C^-1(B^T x0 - g)] gives u_k = x_k (PCG on the Schur system
    # A + B C^-1 B^T with preconditioner P + B C^-1 B^T) and v_k = C^-1(B^T x_k - g).
    rng = np.random.default_rng(8)
    n, r = 12, 4
    Mh = rng.standard_normal((n, n))
    A = Mh @ Mh.T + n * np.eye(n)
    Ph = rng.standard_normal((n, n))
    P = Ph @ Ph.T + np.eye(n)
    Ch = rng.standard_normal((r, r))
    C = Ch @ Ch.T + 0.5 * np.eye(r)
    B = rng.standard_normal((n, r))
    f = rng.standard_normal(n)
    g = rng.standard_normal(r)
    x0 = rng.standard_normal(n)
    Kbig = np.block([[A, B], [B.T, -C]])
    Pbig = np.block([[P, B], [B.T, -C]])
    z0 = np.concatenate([x0, np.linalg.solve(C, B.T @ x0 - g)])
    Ci = np.linalg.inv(C)
    Ks = A + B @ Ci @ B.T
    Ps = P + B @ Ci @ B.T
    fs = f + B @ Ci @ g
    never = lambda rv: False
    _, _, h1 = krylov.pcg(lambda x: Kbig @ x, np.concatenate([f, g]), lambda rv: np.linalg.solve(Pbig, rv), z0, never, 8, keep_x=True)
    _, _, h2 = krylov.pcg(lambda x: Ks @ x, fs, lambda rv: np.linalg.solve(Ps, rv), x0, never, 8, keep_x=True)
    for (r1, z), (r2, x) in zip(h1, h2):
        assert np.allclose(z[:n], x, rtol=1e-8, atol=1e-9)
        assert np.allclose(z[n:], np.linalg.solve(C, B.T @ x - g), rtol=1e-7, atol=1e-8)
        assert np.linalg.norm(r1[n:]) <= 1e-9 * max(1.0, np.linalg.norm(r1))


def test_prop_pcg_iteration_bound():
    # Proposition pcg: ||A x_k - b|| <= eps within ceil(sqrt(k)/2 log(2 sqrt(k) ||r0|| / eps)).
    rng = np.random.default_rng(9)
    n = 60
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, 400.0, n)
    A = (Qm * ev) @ Qm.T
    b = rng.standard_normal(n)
    eps = 1e-9
    x, it, _ = krylov.pcg(lambda x: A @ x, b, lambda rv: rv, np.zeros(n), lambda rv: np.linalg.norm(rv) <= eps, 1000)
    kappa = ev[-1] / ev[0]
    bound = int(np.ceil(0.5 * np.sqrt(kappa) * np.log(2 * np.sqrt(kappa) * np.linalg.norm(b) / eps)))
    assert np.linalg.norm(A @ x - b) <= 10 * eps
    assert it <= bound


def test_preconditioner_inverse_reading():
    # Section 6 block-triangular inverse.  The corrected form
    # [I, -b^-1 AQ; 0, I] diag(b^-1 I, -C^-1) [I, 0; -b^-1 QA, I] inverts the
    # preconditioner for every beta; the printed form agrees only at beta = 1.
    p = small_problem("dense", seed=2)
    X, y, S = ipm_point(p, 3)
    G, d, L = nt.nt_factor(X, S)
    sp = rf.eig_split(G @ G.T, rank_max=3)
    AQ = rf.aq_matrix(p, sp)
    sig = rf.sigma_diag(sp)
    m, dd = AQ.shape
    for beta in (1.0, 2.5):
        P = rf.precond_matrix(AQ, sp, sig, beta)
        Cs = rf.schur_c(AQ, sp, sig, beta)
        Ci = np.linalg.inv(Cs)
        I_m, I_d = np.eye(m), np.eye(dd)
        Z = np.zeros((m, dd))
        corr = (np.block([[I_m, -AQ / beta], [Z.T, I_d]]) @ np.block([[I_m / beta, Z], [Z.T, -Ci]])
                @ np.block([[I_m, Z], [-AQ.T / beta, I_d]]))
        printed = (np.block([[I_m, -AQ], [Z.T, I_d]]) @ np.block([[beta * I_m, Z], [Z.T, -Ci]])
                   @ np.block([[I_m, Z], [-AQ.T, I_d]]))
        Pi = np.linalg.inv(P)
        scale = np.abs(Pi).max()
        assert np.allclose(corr, Pi, atol=1e-9 * scale)
        if beta == 1.0:
            assert np.allclose(printed, Pi, atol=1e-9 * scale)
        else:
            assert not np.allclose(printed, Pi, atol=1e-3 * scale)


@pytest.mark.parametrize("kind", ["dense", "entry"])
def test_beta_rule_in_bracket(kind):
    # Corollary pcg requires lambda_min(A E A^T) <= beta <= lambda_max(A E A^T).
    p = small_problem(kind, seed=4)
    for iters in (1, 5, 9):
        X, y, S = ipm_point(p, iters)
        G, d, L = nt.nt_factor(X, S)
        sp = rf.eig_split(G @ G.T, rank_max=3)
        Am = ops.amat(p)
        ev = np.linalg.eigvalsh(Am @ rf.e_bold(sp) @ Am.T)
        beta = rf.beta_rule(sp, p)
        assert ev[0] <= beta <= ev[-1]


@pytest.mark.parametrize("kind", ["dense", "entry"])
def test_cor_pcg_solve_matches_direct_and_bound(kind):
    # Corollary pcg: indefinite PCG + recovery reproduces the direct Newton step,
    # the bottom residual stays ~0 (Section 6) and the iteration count obeys
    # k <= ceil(1/2 sqrt(cond(A E A^T)) log(cond(A E A^T) ||g|| / (2 eps))).
    p = small_problem(kind, seed=6)
    X, y, S = ipm_point(p, 5)
    G, d, L = nt.nt_factor(X, S)
    W = sym(G @ G.T)
    sp = rf.eig_split(W, rank_max=3)
    res = ipm.residuals(p, X, y, S)
    Ct = sym(res["Rd"] + S)
    bt = res["rp"]
    dX0, dy0, _ = ipm.newton_direct(p, G, ipm.schur_factor(p, G, W), bt, Ct, res["Rd"])
    tol = 1e-12
    dX, dy, info = krylov.solve_newton_pcg(p, sp, bt, Ct, tol=tol)
    assert np.allclose(dX, dX0, rtol=1e-6, atol=1e-7 * np.abs(dX0).max())
    assert np.allclose(dy, dy0, rtol=1e-6, atol=1e-7 * np.abs(dy0).max())
    assert max(info["res_v"]) <= 1e-8 * max(info["res_u"])
    Am = ops.amat(p)
    ev = np.linalg.eigvalsh(Am @ rf.e_bold(sp) @ Am.T)
    cond = ev[-1] / ev[0]
    eps = tol * info["ref"]
    bound = int(np.ceil(0.5 * np.sqrt(cond) * np.log(cond * info["ref"] / (2 * eps))))
    assert info["iterations"] <= bound


def test_minres_solve_matches_direct():
    # Corollary minres: MINRES on eq. augsys (identity preconditioner, x0 = 0) + recovery.
    p = small_problem("dense", seed=12)
    X, y, S = ipm_point(p, 4)
    G, d, L = nt.nt_factor(X, S)
    W = sym(G @ G.T)
    sp = rf.eig_split(W, rank_max=3)
    res = ipm.residuals(p, X, y, S)
    Ct = sym(res["Rd"] + S)
    bt = res["rp"]
    dX0, dy0, _ = ipm.newton_direct(p, G, ipm.schur_factor(p, G, W), bt, Ct, res["Rd"])
    dX, dy, info = krylov.solve_newton_minres(p, sp, bt, Ct, tol=1e-13)
    assert np.allclose(dX, dX0, rtol=1e-6, atol=1e-6 * np.abs(dX0).max())
    assert np.allclose(dy, dy0, rtol=1e-6, atol=1e-6 * np.abs(dy0).max())


def test_rank_rule_and_tau():
    # Experiments section: r = argmax_{i <= rhat} lambda_i / lambda_{i+1}; tau = lambda_{r+1}/2.
    lam = np.array([9.0, 8.0, 0.5, 0.4, 0.3, 0.2])
    Qm = np.eye(6)
    W = np.diag(lam)
    sp = rf.eig_split(W, rank_max=4)
    assert sp["r"] == 2
    assert sp["tau"] == 0.25
    assert rf.dim_d(6, 2) == 11
    sp1 = rf.eig_split(W, rank_fixed=3)
    assert sp1["r"] == 3 and sp1["tau"] == 0.2
    # eigenvector signs: largest-magnitude entry positive
    assert np.all(sp["V"].max(axis=0) >= -sp["V"].min(axis=0))
