"""GPU parity at late interior-point iterates (mu ~ 1e-7), where the
safeguards of the preconditioner solve matter and the small eigenvalues of W
cluster.

Points: the oracle's own iterates of the Gaussian sensing workload n = 20
(iterations 10 and 11: mu = 6.4e-7, 5.3e-8) and of a small completion
instance (iteration 8: mu = 3.7e-7).  There X and S are so ill-conditioned
that the scaling point W itself is determined only to about eps cond(X)
relative (the two sides' eigenvalues of W differ by up to 1e-7 relative:
the oracle forms W and diagonalises it, absolute accuracy eps ||W||; the
GPU runs Jacobi on the factor).  So:

* the GPU's scaling is judged by its defining property W S W = X (Nesterov-
  Todd, Introduction), no worse than the oracle's own factor at that point;
* sdp_newton_apply (eq. augsys, Section 5 products) and sdp_precond_apply
  (Section 6) are compared with the oracle evaluated on the GPU's own
  eigen-split (lam, V from sdp_get_scaling): same point, same basis, so every
  block is compared entry by entry (operator) or by the normwise backward
  error of P z = x (preconditioner), as at the early iterates;
* sdp_inner_solve (eq. Newt-eps) by the residuals of its two equations at
  the GPU's own scaling point: the primal one to the inner tolerance, the
  NT-scaled second one to 1e-8 or ten times what the direct Schur-complement
  solve reaches at the same point, whichever is larger (1e-8 to 5e-8 at these
  mu: the rounding floor of that equation, not a property of either method).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import ipm, nt, operators as ops, reform as rf  # noqa: E402
from paper_2407_14013_amd import Context  # noqa: E402

CASES = [("cfg0", 10), ("cfg0", 11), ("entry", 8)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def problem(which):
    return workloads.config(0) if which == "cfg0" else workloads.matrix_completion(16, 2, 100, seed=3)


def late_point(which, iters):
    p = problem(which)
    res = ipm.solve(p, maxit=iters)
    assert res["status"] == "maxit"  # still an interior iterate, not the final one
    return p, res["X"], res["y"], res["S"]


def split_of(X, S):
    G, d, L = nt.nt_factor(X, S)
    return rf.eig_split(G @ G.T)


def gpu_split(g, n):
    """The oracle's split dictionary built from the GPU's eigenvalues and eigenvectors."""
    lam, V, r = g["lam"], host(g["V"]), g["r"]
    return {"n": n, "r": r, "tau": 0.5 * lam[r], "lam": lam, "V": V, "Q": V[:, :r], "Qp": V[:, r:],
            "lam_top": lam[:r], "lam_perp": lam[r:]}


@pytest.mark.parametrize("which,iters", CASES)
def test_operator_at_late_iterate(which, iters):
    p, X, y, S = late_point(which, iters)
    m, n = p["m"], p["n"]
    mu = float(np.sum(X * S)) / n
    G, _, _ = nt.nt_factor(X, S)
    Wo = G @ G.T
    rng = np.random.default_rng(iters)
    with Context(p) as ctx:
        ctx.set_point(dev(X), dev(y), dev(S))
        g = ctx.get_scaling()
        sp = gpu_split(g, n)
        N = ctx.aug_dim()
        assert g["r"] == split_of(X, S)["r"] and N == m + rf.dim_d(n, sp["r"])
        E = rf.e_matrix(sp)
        sig = rf.sigma_diag(sp)
        errs = []
        for trial in range(3):
            x = rng.standard_normal(N)
            if trial == 1:
                x[m:] = 0.0  # u only
            if trial == 2:
                x[:m] = 0.0  # v only
            got = host(ctx.newton_apply(dev(x)))
            t, b = rf.aug_apply(p, sp, E, sig, x[:m], x[m:])
            ref = np.concatenate([t, b])
            errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    # W S W = X for the GPU's W and for the oracle's
    Wg = (sp["V"] * sp["lam"]) @ sp["V"].T
    res_g = np.linalg.norm(Wg @ S @ Wg - X) / np.linalg.norm(X)
    res_o = np.linalg.norm(Wo @ S @ Wo - X) / np.linalg.norm(X)
    print(f"{which} it {iters} (mu {mu:.1e}): operator errors {', '.join(f'{e:.1e}' for e in errs)}; "
          f"|WSW - X|/|X| GPU {res_g:.1e} oracle {res_o:.1e}")
    assert max(errs) <= 1e-10
    assert res_g <= max(10.0 * res_o, 1e-13)


@pytest.mark.parametrize("which,iters", CASES)
def test_precond_at_late_iterate(which, iters):
    p, X, y, S = late_point(which, iters)
    m, n = p["m"], p["n"]
    rng = np.random.default_rng(100 + iters)
    with Context(p) as ctx:
        ctx.set_point(dev(X), dev(y), dev(S))
        g = ctx.get_scaling()
        sp = gpu_split(g, n)
        sig = rf.sigma_diag(sp)
        beta = rf.beta_rule(sp, p)
        assert abs(g["beta"] - beta) <= 1e-10 * beta
        P = rf.precond_matrix(rf.aq_matrix(p, sp), sp, sig, beta)
        normP = np.linalg.norm(P, 2)
        N = ctx.aug_dim()
        assert N == P.shape[0]
        for trial in range(2):
            x = rng.standard_normal(N)
            if trial == 1:
                x[m:] = 0.0  # f only
            z = host(ctx.precond_apply(dev(x)))
            bwd = np.linalg.norm(P @ z - x) / (normP * np.linalg.norm(z) + np.linalg.norm(x))
            print(f"{which} it {iters} trial {trial}: backward error {bwd:.1e}")
            assert bwd <= 1e-10


@pytest.mark.parametrize("sampled", [0, 1])
@pytest.mark.parametrize("which,iters", CASES)
def test_inner_solve_at_late_iterate(which, iters, sampled):
    if sampled and which != "entry":
        pytest.skip("the sampled form applies to entry-sampling constraints")
    p, X, y, S = late_point(which, iters)
    r = ipm.residuals(p, X, y, S)
    Ct = r["Rd"] + S
    bt = r["rp"]
    with Context(p, sparse_sandwich=sampled) as ctx:
        ctx.set_point(dev(X), dev(y), dev(S))
        dX, dy, st = ctx.inner_solve(dev(bt), dev(Ct))
        g = ctx.get_scaling()
    dX, dy = host(dX), host(dy)
    # the Newton system is the one at the solver's own scaling point W = G G^T
    V = host(g["V"])
    G = V * np.sqrt(g["lam"])
    W = G @ G.T
    scale = np.linalg.norm(bt + ops.a_op(p, W @ Ct @ W))
    e_primal = np.linalg.norm(ops.a_op(p, dX) - bt) / scale
    Gi = np.linalg.inv(G)
    rhs = G.T @ (ops.at_op(p, dy) - Ct) @ G
    e_second = np.linalg.norm(Gi @ dX @ Gi.T - rhs) / np.linalg.norm(rhs)
    # the second equation's attainable accuracy at this mu: what the direct
    # Schur-complement solve (the oracle's method) reaches, in its own scaling
    Go, _, _ = nt.nt_factor(X, S)
    Wo = Go @ Go.T
    dXo, dyo, _ = ipm.newton_direct(p, Go, ipm.schur_factor(p, Go, Wo), bt, Ct, r["Rd"])
    Goi = np.linalg.inv(Go)
    rhs_o = Go.T @ (ops.at_op(p, dyo) - Ct) @ Go
    e_direct = np.linalg.norm(Goi @ dXo @ Goi.T - rhs_o) / np.linalg.norm(rhs_o)
    print(f"{which} it {iters} sampled {sampled}: pcg {st['iterations']} rel_res {st['rel_res']:.1e} "
          f"primal {e_primal:.1e} second {e_second:.1e} (direct solve: {e_direct:.1e})")
    assert st["converged"] == 1 and st["rel_res"] <= 1e-10
    assert e_primal <= 1e-9 and e_second <= max(1e-8, 10.0 * e_direct)
