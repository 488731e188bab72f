"""Pins for the oracle's nonnegative-orthant (LP) block (eq. rmc-sdp, eq. snl-sdp).

* A diagonal SDP with an LP block is a linear program in (diag X, x): the
  oracle IPM's optimum must equal SciPy's HiGHS optimum of that LP.
* The direct Newton solve with the LP block satisfies the unsubstituted
  KKT system of eq. Newt-eps extended by B x, and its factor gives
  M = A (W (x)_s W) A^T + B diag(w^2) B^T written out entry by entry.
* The LP split reproduces diag(w^2) = tau^2 E_lp + P_T Sigma_lp^{-1} P_T^T
  exactly, with or without the cap on |T|.
* The augmented operator with the LP block equals its explicit matrix, and
  solving that system exactly and recovering gives the direct Newton step.
* beta with the LP block stays inside the bracket of Corollary pcg for the
  (1,1) block A E A^T + B diag(e2) B^T.
* The whole method: the PCG-based IPM reaches the direct IPM's point; RMC
  recovers X* (the paper's Table rmc reports exact recovery) and its LP
  part equals the l1 misfit of eq. rmc; SNL recovers the sensor positions
  with a rank-d solution (Table snl).
"""
import numpy as np
import pytest
from scipy.optimize import linprog

import workloads
from oracle import certify, ipm, krylov, nt, operators as ops, reform as rf
from oracle.notation import sym


def diagonal_with_lp(seed, n=4, m=3, ell=5):
    """Diagonal A_i and C plus an LP block with a dense random B: an LP in (diag X, x)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 2.0, size=(m, n))
    B = rng.uniform(-1.0, 1.0, size=(m, ell))
    z_feas = rng.uniform(0.5, 1.5, size=n + ell)
    b = np.hstack([a, B]) @ z_feas
    c_sdp = rng.uniform(0.5, 2.0, size=n)
    c_lp = rng.uniform(0.5, 2.0, size=ell)
    A = np.stack([np.diag(a[i]).reshape(-1) for i in range(m)])
    lp = {"ptr": np.arange(0, m * ell + 1, m, dtype=np.int64),
          "row": np.tile(np.arange(m, dtype=np.int32), ell),
          "val": B.T.reshape(-1).copy(), "c": c_lp}
    p = {"kind": "dense", "n": n, "m": m, "A": A, "b": b, "C": np.diag(c_sdp), "lp": lp}
    return p, np.hstack([a, B]), np.concatenate([c_sdp, c_lp])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_diagonal_sdp_with_lp_matches_highs(seed):
    p, Aeq, cost = diagonal_with_lp(seed)
    assert np.allclose(ops.b_matrix(p), Aeq[:, p["n"]:])
    ref = linprog(cost, A_eq=Aeq, b_eq=p["b"], bounds=(0, None), method="highs")
    assert ref.status == 0
    res = ipm.solve(p)
    assert res["status"] == "converged"
    c = certify.certificate(p, res["X"], res["y"], res["S"], res["x"], res["s"])
    assert c["pinf"] <= 1e-8 and c["dinf"] <= 1e-8 and c["relgap"] <= 1e-8
    assert c["min_x"] > 0 and c["min_s"] > 0 and c["lmin_X"] > 0 and c["lmin_S"] > 0
    assert abs(c["pobj"] - ref.fun) <= 1e-7 * (1.0 + abs(ref.fun))


def rmc_point(iters, seed=3):
    p = workloads.robust_completion(8, 24, 2, seed=seed)
    res = ipm.solve(p, maxit=iters)
    return p, res


def test_direct_newton_with_lp_solves_unsubstituted_system():
    p, res = rmc_point(3)
    X, y, S, x, s = res["X"], res["y"], res["S"], res["x"], res["s"]
    G, _, _ = nt.nt_factor(X, S)
    W = sym(G @ G.T)
    w = np.sqrt(x / s)
    r = ipm.residuals(p, X, y, S, x, s)
    rng = np.random.default_rng(2)
    n, m, ell = p["n"], p["m"], x.size
    Ct = sym(rng.standard_normal((n, n)))
    ct = rng.standard_normal(ell)
    bt = rng.standard_normal(m)
    fac = ipm.schur_factor(p, G, W, w)
    dX, dy, dS, dx, ds = ipm.newton_direct(p, G, fac, bt, Ct, r["Rd"], (w, ct, r["rd"]))
    B = ops.b_matrix(p)
    assert np.allclose(ops.a_op(p, dX) + B @ dx, bt, atol=1e-10 * np.abs(bt).max())
    assert np.allclose(ops.at_op(p, dy) + dS, r["Rd"], atol=1e-12)
    assert np.allclose(B.T @ dy + ds, r["rd"], atol=1e-12)
    rhs = W @ (r["Rd"] - Ct) @ W
    assert np.allclose(dX + W @ dS @ W, rhs, atol=1e-9 * np.abs(rhs).max())
    rhs_lp = w * w * (r["rd"] - ct)
    assert np.allclose(dx + w * w * ds, rhs_lp, atol=1e-9 * np.abs(rhs_lp).max())
    # M_ij = <A_i, W A_j W> + sum_k B_ik w_k^2 B_jk, entry by entry
    A = [ops.a_matrix(p, i) for i in range(m)]
    M = np.array([[np.sum(A[i] * (W @ A[j] @ W)) + sum(B[i, k] * w[k] ** 2 * B[j, k] for k in range(ell))
                   for j in range(m)] for i in range(m)])
    _, _, R = fac
    assert np.allclose(R.T @ R, M, rtol=1e-10, atol=1e-12 * np.abs(M).max())
    assert np.allclose(ipm.schur_matrix(p, G, W, w), M, rtol=1e-12, atol=1e-13 * np.abs(M).max())


@pytest.mark.parametrize("cap", [None, 3])
def test_lp_split_identity(cap):
    rng = np.random.default_rng(4)
    sp = {"tau": 0.7}
    w = np.exp(rng.uniform(-3.0, 3.0, size=40))
    lsp = rf.lp_split(sp, w, cap=cap)
    T = lsp["T"]
    above = np.flatnonzero(w > 1.4)
    if cap is None:
        assert np.array_equal(T, above)
    else:
        assert T.size == 3 and np.array_equal(T, np.sort(above[np.argsort(-w[above])[:3]]))
    D = lsp["e2"] * 0.49
    D[T] += 1.0 / lsp["sig"]
    assert np.allclose(D, w * w, rtol=1e-14)
    assert np.all(lsp["sig"] > 0)
    off = np.setdiff1d(np.arange(w.size), T)
    if cap is None:
        assert np.all(lsp["e2"][off] <= 4.0)


def test_lp_split_cap_keeps_or_drops_tied_groups_whole():
    sp = {"tau": 0.1}
    w = np.array([5.0, 1.0, 5.0, 7.0, 5.0, 0.05])
    assert list(rf.lp_split(sp, w, cap=3)["T"]) == [3]
    assert list(rf.lp_split(sp, w, cap=4)["T"]) == [0, 2, 3, 4]
    assert list(rf.lp_split(sp, w, cap=10)["T"]) == [0, 1, 2, 3, 4]


def rmc_split(iters):
    p, res = rmc_point(iters)
    G, _, _ = nt.nt_factor(res["X"], res["S"])
    sp = rf.eig_split(sym(G @ G.T), rank_max=3)
    lsp = rf.lp_split(sp, np.sqrt(res["x"] / res["s"]))
    return p, res, G, sp, lsp


def test_aug_apply_lp_matches_explicit():
    p, _, _, sp, lsp = rmc_split(6)
    assert lsp["t"] > 0
    K = rf.aug_matrix_lp(p, sp, lsp)
    assert K.shape[0] == p["m"] + rf.dim_d(p["n"], sp["r"]) + lsp["t"]
    x = np.random.default_rng(5).standard_normal(K.shape[0])
    t, b = rf.aug_apply_lp(p, sp, lsp, rf.e_matrix(sp), rf.sigma_diag(sp), x[: p["m"]], x[p["m"]:])
    ref = K @ x
    assert np.allclose(np.concatenate([t, b]), ref, atol=1e-11 * np.abs(ref).max())
    assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())


@pytest.mark.parametrize("iters", [2, 6, 10])
def test_augrec_lp_equals_direct_newton(iters):
    p, res, G, sp, lsp = rmc_split(iters)
    X, y, S, x, s = res["X"], res["y"], res["S"], res["x"], res["s"]
    W = sym(G @ G.T)
    w = np.sqrt(x / s)
    r = ipm.residuals(p, X, y, S, x, s)
    Ct, ct, bt = sym(r["Rd"] + S), r["rd"] + s, r["rp"]
    dX0, dy0, _, dx0, _ = ipm.newton_direct(p, G, ipm.schur_factor(p, G, W, w), bt, Ct, r["Rd"], (w, ct, r["rd"]))
    E = rf.e_matrix(sp)
    gu, gv = rf.aug_rhs_lp(p, sp, lsp, E, bt, Ct, ct)
    sol = np.linalg.solve(rf.aug_matrix_lp(p, sp, lsp), np.concatenate([gu, gv]))
    dX, dy, dx = rf.recover_lp(p, sp, lsp, E, sol[: p["m"]], sol[p["m"]:], Ct, ct)
    for a, b_ in ((dX, dX0), (dy, dy0), (dx, dx0)):
        assert np.allclose(a, b_, rtol=1e-7, atol=1e-8 * np.abs(b_).max())


@pytest.mark.parametrize("which", ["rmc", "snl"])
def test_beta_rule_lp_in_bracket(which):
    # Corollary pcg asks for lambda_min <= beta <= lambda_max of the (1,1) block
    # of eq. augsys, which with the LP block is A E A^T + B diag(e2) B^T.
    if which == "rmc":
        p = workloads.robust_completion(12, 60, 3, seed=6)
    else:
        p = workloads.sensor_localization(8, 20, 6, 2, 1, seed=5, kind="sparse")
    Am, B = ops.amat(p), ops.b_matrix(p)
    raised = 0
    for iters in (2, 6, 10, 14):
        res = ipm.solve(p, maxit=iters)
        G, _, _ = nt.nt_factor(res["X"], res["S"])
        sp = rf.eig_split(sym(G @ G.T), rank_max=3)
        lsp = rf.lp_split(sp, np.sqrt(res["x"] / res["s"]))
        H = Am @ rf.e_bold(sp) @ Am.T + B @ np.diag(lsp["e2"]) @ B.T
        ev = np.linalg.eigvalsh(H)
        beta = rf.beta_rule_lp(sp, lsp, p)
        assert ev[0] <= beta <= ev[-1] * (1 + 1e-12)
        assert beta >= rf.beta_rule(sp, p)
        raised += beta > rf.beta_rule(sp, p)
    assert raised > 0  # the LP term decides beta somewhere on the path


def pcg_newton(problem, X, S, G, d, W, bt, Ct, Rd, lp=None):
    x, s, w, ct, rd = lp
    sp = rf.eig_split(W)
    lsp = rf.lp_split(sp, w)
    dX, dy, dx, _ = krylov.solve_newton_pcg_lp(problem, sp, lsp, bt, Ct, ct, tol=1e-10, maxit=3000)
    return dX, dy, sym(Rd - ops.at_op(problem, dy)), dx, rd - ops.bt_op(problem, dy)


def test_ipm_with_reformulated_newton_and_lp_reaches_same_solution():
    p = workloads.robust_completion(12, 60, 3, seed=6)
    ref = ipm.solve(p)
    got = ipm.solve(p, newton=pcg_newton)
    assert ref["status"] == got["status"] == "converged"
    assert np.linalg.norm(got["X"] - ref["X"]) <= 1e-7 * np.linalg.norm(ref["X"])
    assert np.linalg.norm(got["x"] - ref["x"]) <= 1e-6 * (1.0 + np.linalg.norm(ref["x"]))


def test_rmc_recovers_planted_matrix_and_l1_misfit():
    p = workloads.robust_completion(30, 300, 5, seed=1)
    res = ipm.solve(p)
    c = certify.certificate(p, res["X"], res["y"], res["S"], res["x"], res["s"])
    assert res["status"] == "converged"
    assert c["pinf"] <= 1e-8 and c["dinf"] <= 1e-8 and c["relgap"] <= 1e-8 and c["min_x"] > 0 and c["min_s"] > 0
    err = np.linalg.norm(res["X"] - p["Xstar"]) / np.linalg.norm(p["Xstar"])
    assert err <= 1e-6
    # eq. rmc: at the optimum the LP part is the l1 misfit of P_m svec(X) against b
    m = p["m"]
    v, w = res["x"][:m], res["x"][m:]
    jk = p["jk"]
    kappa = np.where(jk[:, 0] == jk[:, 1], 1.0, np.sqrt(2.0))
    misfit = np.abs(kappa * (res["X"][jk[:, 0], jk[:, 1]] - p["b"])).sum()
    assert abs(v.sum() + w.sum() - misfit) <= 1e-6 * misfit
    # the misfit is carried by the outliers
    assert set(np.flatnonzero(np.abs(v - w) > 1e-3).tolist()) <= set(p["outliers"].tolist())


def test_snl_recovers_sensor_positions():
    q = workloads.sensor_localization(20, 120, 30, 3, 1, seed=2)
    res = ipm.solve(q)
    c = certify.certificate(q, res["X"], res["y"], res["S"], res["x"], res["s"])
    assert res["status"] == "converged"
    assert c["pinf"] <= 1e-8 and c["dinf"] <= 1e-8 and c["relgap"] <= 1e-8
    d = q["d"]
    assert np.allclose(res["X"][:d, :d], np.eye(d), atol=1e-8)
    assert np.linalg.norm(res["X"][:d, d:] - q["Ystar"]) <= 1e-6
    lam = np.linalg.eigvalsh(res["X"])
    assert lam[-d - 1] <= 1e-6 * lam[-1]


def test_certificate_with_lp_detects_planted_mistakes():
    p = workloads.robust_completion(12, 60, 3, seed=6)
    res = ipm.solve(p)
    good = certify.certificate(p, res["X"], res["y"], res["S"], res["x"], res["s"])
    x_bad = res["x"].copy()
    x_bad[0] += 1.0
    bad_p = certify.certificate(p, res["X"], res["y"], res["S"], x_bad, res["s"])
    s_bad = res["s"].copy()
    s_bad[1] += 10.0
    bad_d = certify.certificate(p, res["X"], res["y"], res["S"], res["x"], s_bad)
    assert good["pinf"] <= 1e-8 and bad_p["pinf"] > 1e-5
    assert good["dinf"] <= 1e-8 and bad_d["dinf"] > 1e-5


@pytest.mark.slow
@pytest.mark.parametrize("which", ["rmc", "snl"])
def test_pcg_counts_bounded_on_fig_thm_instances(which):
    # Fig. thm / Corollary pcg on the experiments' own small instances
    # (RMC n=50, m=1200, m_o=20; SNL n=50, m=1300, m_o=25): PCG to the paper's
    # 1e-6 on every Newton system of the oracle's trajectory needs no more
    # iterations once mu < 1e-3 than it did while 1e-3 <= mu <= 1, and the
    # low-rank LP part settles on the outliers.
    if which == "rmc":
        p, m_o = workloads.robust_completion(50, 1200, 20, seed=7), 20
    else:
        p, m_o = workloads.sensor_localization(50, 1150, 150, 22, 3, seed=8), 25
    rows = []

    def newton(problem, X, S, G, d, W, bt, Ct, Rd, lp=None):
        x, s, w, ct, rd = lp
        sp = rf.eig_split(W)
        lsp = rf.lp_split(sp, w)
        _, _, _, info = krylov.solve_newton_pcg_lp(problem, sp, lsp, bt, Ct, ct, tol=1e-6, maxit=3000)
        mu = (np.sum(X * S) + x @ s) / (problem["n"] + x.size)
        rows.append((mu, info["iterations"], lsp["t"]))
        return ipm.newton_direct(problem, G, ipm.schur_factor(problem, G, W, w), bt, Ct, Rd, (w, ct, rd))

    res = ipm.solve(p, newton=newton)
    assert res["status"] == "converged"
    early = max(k for mu, k, _ in rows if 1e-3 <= mu <= 1.0)
    late = max(k for mu, k, _ in rows if mu < 1e-3)
    assert late <= early, (early, late)
    assert min(mu for mu, _, _ in rows) < 1e-6
    assert rows[-1][2] == m_o
