"""Theory validation on the GPU path (Theorem main, Corollary pcg; the
experiment behind the paper's Fig. thm).

* At every Newton system of the oracle's trajectory on the Gaussian sensing
  workload n = 20 (predictor and corrector of each iteration, mu from 6e2
  down to 5e-8), the GPU's indefinite PCG to the paper's inner tolerance
  1e-6 is run on the same system and its iteration count compared with the
  oracle's PCG (the same method -- Definition pcg, the Section 6
  preconditioner, the same beta -- in another arithmetic): within a factor
  1.5 plus 5 iterations, and bounded as mu -> 0 (the systems at mu < 1e-3
  need no more iterations than those at 1e-3 <= mu <= 1).
* Along the GPU's own trajectories (sdp_ipm_step at the default inner
  tolerance 1e-10) on the n = 20 and n = 200 workloads, the predictor and
  corrector counts of the late iterations (mu < 1e-3) stay within those of
  the iterations where the rank has settled (1e-3 <= mu <= 1), so the cost
  per Newton system does not grow with 1/mu.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import ipm, krylov, reform as rf  # noqa: E402
from paper_2407_14013_amd import Context  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def oracle_systems(p):
    rows = []

    def newton(problem, X, S, G, d, W, bt, Ct, Rd):
        sp = rf.eig_split(W)
        _, _, info = krylov.solve_newton_pcg(problem, sp, bt, Ct, tol=1e-6, maxit=2000)
        rows.append({"mu": float(np.sum(X * S)) / problem["n"], "X": X.copy(), "S": S.copy(), "bt": bt.copy(),
                     "Ct": Ct.copy(), "pcg": int(info["iterations"])})
        return ipm.newton_direct(problem, G, ipm.schur_factor(problem, G, W), bt, Ct, Rd)

    res = ipm.solve(p, newton=newton)
    assert res["status"] == "converged"
    return rows


def test_gpu_pcg_counts_track_the_oracle_along_its_trajectory():
    p = workloads.config(0)
    rows = oracle_systems(p)
    got = []
    with Context(p, inner_tol=1e-6) as ctx:
        for r in rows:
            ctx.set_point(dev(r["X"]), dev(np.zeros(p["m"])), dev(r["S"]))
            _, _, st = ctx.inner_solve(dev(r["bt"]), dev(r["Ct"]))
            assert st["converged"] == 1
            got.append(st["iterations"])
    for r, g in zip(rows, got):
        print(f"mu {r['mu']:.2e}: oracle pcg {r['pcg']:4d}  gpu pcg {g:4d}")
        assert g <= 1.5 * r["pcg"] + 5, (r["mu"], r["pcg"], g)
    early = max(g for r, g in zip(rows, got) if 1e-3 <= r["mu"] <= 1.0)
    late = max(g for r, g in zip(rows, got) if r["mu"] < 1e-3)
    assert late <= early, (early, late)
    assert min(r["mu"] for r in rows) < 1e-7


@pytest.mark.parametrize("cfg", [0, 1])
def test_gpu_trajectory_pcg_counts_stay_bounded(cfg):
    p = workloads.config(cfg)
    traj = []
    with Context(p) as ctx:
        for _ in range(100):
            st = ctx.ipm_step()
            if st["converged"]:
                break
            traj.append((st["mu"], st["pcg_pred"], st["pcg_corr"]))
    for mu, a, b in traj:
        print(f"config {cfg} mu {mu:.2e}: predictor {a:3d} corrector {b:3d}")
    early = max(max(a, b) for mu, a, b in traj if 1e-3 <= mu <= 1.0)
    late = max(max(a, b) for mu, a, b in traj if mu < 1e-3)
    assert min(mu for mu, _, _ in traj) < 1e-6
    assert late <= early, (early, late)
