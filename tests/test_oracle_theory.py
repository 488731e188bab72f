"""Theory validation along an interior-point trajectory (Theorem main,
Corollary pcg; the experiment of the paper's Fig. thm, on the Gaussian sensing
workload n = 20, r = 2, m = 120 instead of RMC / SNL).

At every iterate of the oracle's interior-point method the test forms

* the Schur complement M = script-A (W kron_s W) script-A^T of the Newton
  system (eq. Newt-eps), whose condition number grows like 1/mu (to the limit
  of FP64),
* the augmented matrix of eq. augsys from the eigen-split of W, whose
  condition number the theorem bounds independently of mu, and
* the number of indefinite-PCG iterations (Corollary pcg, preconditioner of
  Section 6) that reach the paper's inner tolerance 1e-6 on the Newton
  system at that iterate.

Pins: cond(M) grows by more than twelve orders of magnitude while cond(augsys)
stays within a factor 10 once the rank r is identified (mu <= 1), and the PCG
count does not grow as mu -> 0.
"""
import numpy as np

import workloads
from oracle import ipm, krylov, reform as rf


def trajectory():
    p = workloads.config(0)
    rows = []

    def newton(problem, X, S, G, d, W, bt, Ct, Rd):
        fac = ipm.schur_factor(problem, G, W)
        M = ipm.schur_matrix(problem, G, W)
        sp = rf.eig_split(W)
        sv = np.linalg.svd(rf.aug_matrix(problem, sp), compute_uv=False)
        _, _, info = krylov.solve_newton_pcg(problem, sp, bt, Ct, tol=1e-6, maxit=2000)
        mu = float(np.sum(X * S) / problem["n"])
        rows.append({"mu": mu, "cond_M": float(np.linalg.cond(M)), "cond_K": float(sv[0] / sv[-1]),
                     "pcg": int(info["iterations"]), "r": int(sp["r"])})
        return ipm.newton_direct(problem, G, fac, bt, Ct, Rd)

    res = ipm.solve(p, newton=newton)
    assert res["status"] == "converged"
    return rows


def test_augmented_system_stays_well_conditioned_while_newton_system_does_not():
    rows = trajectory()
    first, last = rows[0], rows[-1]
    assert last["mu"] < 1e-7
    assert last["cond_M"] >= 1e12 * first["cond_M"] and last["cond_M"] >= 1e15
    settled = [r for r in rows if r["mu"] <= 1.0]
    assert len(settled) >= 8 and all(r["r"] == 2 for r in settled)
    ck = [r["cond_K"] for r in settled]
    assert max(ck) <= 10.0 * min(ck), ck
    # bounded PCG iterations independent of 1/mu: the late systems need no more
    # than the ones at mu ~ 1
    early = max(r["pcg"] for r in settled if r["mu"] >= 1e-3)
    late = max(r["pcg"] for r in settled if r["mu"] < 1e-3)
    assert late <= early, (early, late)
    assert max(r["pcg"] for r in rows) <= 200
