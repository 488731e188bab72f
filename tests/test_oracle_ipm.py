"""Pins for the oracle interior-point method (brute force, closed forms, certificates)."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import brute, certify, ipm, krylov, reform as rf
from oracle.notation import sym

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "brute_optima.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def check_certificate(p, res, tol=1e-8):
    c = certify.certificate(p, res["X"], res["y"], res["S"])
    assert res["status"] == "converged"
    assert c["pinf"] <= tol and c["dinf"] <= tol and c["relgap"] <= tol
    assert c["lmin_X"] > 0 and c["lmin_S"] > 0
    return c


def test_lp_reduction_matches_enumeration(golden):
    for case in golden["lp_diagonal"]["cases"]:
        q = brute.lp_instance(case["n"], case["m"], case["seed"])
        res = ipm.solve(q)
        check_certificate(q, res)
        pobj = float(np.sum(q["C"] * res["X"]))
        assert abs(pobj - case["optimum"]) <= 1e-7 * (1 + abs(case["optimum"]))
        assert np.allclose(np.diag(res["X"]), case["x"], atol=1e-5)


def test_two_by_two_closed_form(golden):
    for case in golden["two_by_two"]["cases"]:
        q = brute.two_by_two_instance(case["seed"])
        res = ipm.solve(q)
        check_certificate(q, res)
        pobj = float(np.sum(q["C"] * res["X"]))
        assert abs(pobj - case["optimum"]) <= 1e-7 * (1 + abs(case["optimum"]))
        assert np.allclose(res["X"], case["X"], atol=1e-4)


def test_determined_system(golden):
    for case in golden["determined"]["cases"]:
        q = brute.determined_instance(case["n"], case["seed"])
        res = ipm.solve(q)
        check_certificate(q, res)
        Xg = np.array(case["X"])
        assert np.linalg.norm(res["X"] - Xg) <= 1e-6 * np.linalg.norm(Xg)


def test_config0_planted_recovery_and_certificate():
    # Trace minimisation recovers the planted rank-r X* = U U^T (unique low-rank
    # solution assumed in eq. sdp-asm-p); the final iterate is centred (Assumption 1).
    p = workloads.config(0)
    res = ipm.solve(p)
    c = check_certificate(p, res)
    Xs = p["U"] @ p["U"].T
    assert np.linalg.norm(res["X"] - Xs) <= 1e-6 * np.linalg.norm(Xs)
    assert abs(c["pobj"] - np.trace(Xs)) <= 1e-8 * np.trace(Xs)
    assert c["delta"] < 1.0
    # W's eigenvalues split into r* = 2 large and n - r* small ones (Lemma eigsplit)
    from oracle import nt
    G, d, L = nt.nt_factor(res["X"], res["S"])
    w = np.linalg.eigvalsh(G @ G.T)[::-1]
    assert w[1] / w[2] > 1e3


def test_planted_recovery_entry_sampling():
    p = workloads.matrix_completion(12, 2, 50, seed=3)
    res = ipm.solve(p)
    check_certificate(p, res)
    Xs = p["U"] @ p["U"].T
    assert np.linalg.norm(res["X"] - Xs) <= 1e-6 * np.linalg.norm(Xs)


def reformulated_newton(problem, X, S, G, d, W, bt, Ct, Rd):
    sp = rf.eig_split(W, rank_max=10)
    dX, dy, _ = krylov.solve_newton_pcg(problem, sp, bt, Ct, tol=1e-12, maxit=2000)
    from oracle import operators as ops
    return dX, dy, sym(Rd - ops.at_op(problem, dy))


def test_ipm_with_reformulated_newton_reaches_same_solution():
    # Corollary pcg inside the IPM: same optimum as the direct Schur solve.
    p = workloads.config(0)
    direct = ipm.solve(p)
    ref = ipm.solve(p, newton=reformulated_newton)
    check_certificate(p, ref)
    assert abs(ref["history"][-1]["pobj"] - direct["history"][-1]["pobj"]) <= 1e-8 * abs(direct["history"][-1]["pobj"])
    assert np.linalg.norm(ref["X"] - direct["X"]) <= 1e-6 * np.linalg.norm(direct["X"])


def test_certificate_detects_planted_mistakes():
    # A wrong dual (a flipped sign of y) or a perturbed X must fail the certificate.
    p = workloads.config(0)
    res = ipm.solve(p)
    good = certify.certificate(p, res["X"], res["y"], res["S"])
    bad_y = certify.certificate(p, res["X"], -res["y"], res["S"])
    assert bad_y["dinf"] > 1e-3 and good["dinf"] < 1e-8
    Xp = res["X"].copy()
    Xp[0, 1] += 1e-3
    Xp[1, 0] += 1e-3
    assert certify.certificate(p, Xp, res["y"], res["S"])["pinf"] > 1e-6
