"""GPU checks of sdp_adjoint and the differentiable layer (paper_2407_14013_amd/layer.py).

sdp_adjoint returns the derivative of the central-path point at the current
mu (after re-centring), i.e. the self-adjoint Newton KKT system of eq.
Newt-eps solved with C~ = dL/dX, b~ = 0.  Checked on the Gaussian sensing
workload (n = 20, m = 120), whose problems are strictly feasible on both sides:

* against the oracle's gradient from the same interior point (both re-centre
  to a distance <= 1e-8 and solve the same KKT system).  The gradient solve
  runs at inner_tol 1e-13: at 1e-10 the reformulated solve (the oracle's own
  PCG as much as the GPU's) leaves a 7e-4 relative error in the gradient at
  mu ~ 1e-2, 1e-6 at 1e-12.  Checked element-wise at 1e-5 there, and by the
  KKT residuals of the returned gradient (A(dL/dC) = 0 and, NT-scaled,
  dL/dC = W (A^T(dL/db) - dL/dX) W) at smaller mu, where the system is too
  ill-conditioned for element-wise agreement;
* against central finite differences of central-path points computed by the
  GPU itself for perturbed data at the same mu;
* with the FP32 inner operator (the refinement brings the solve to the FP64
  tolerance), and through torch autograd.

The generic-data checks of the solution-map derivative (envelope theorem,
finite differences of full solves) live with the oracle: such problems have
m below the tangent dimension, where the reformulated system the GPU solves
is not well conditioned.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import adjoint as oadj, ipm, nt, operators as ops  # noqa: E402
from paper_2407_14013_amd import Context, SdpError  # noqa: E402
from paper_2407_14013_amd import _lib as L  # noqa: E402
from paper_2407_14013_amd.layer import SDPLayer  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def target_of(n, seed=11):
    V = np.random.default_rng(seed).standard_normal((n, 2))
    return V @ V.T


@pytest.mark.parametrize("prec", [L.SDP_PREC_F64, L.SDP_PREC_F32])
@pytest.mark.parametrize("tol", [1e-2, 1e-4])
def test_adjoint_matches_oracle_gradient(tol, prec):
    p = workloads.config(0)
    res = ipm.solve(p, tol=tol)
    X, y, S = res["X"], res["y"], res["S"]
    GX = 2.0 * (X - target_of(p["n"]))
    gC0, gb0 = oadj.solution_gradient(p, X, y, S, GX)
    with Context(p, inner_prec=prec, inner_tol=1e-13) as ctx:
        ctx.set_point(dev(X), dev(y), dev(S))
        gb, gC, st = ctx.adjoint(dev(GX))
        Xc, yc, Sc = (host(t) for t in ctx.get_point())
    gb, gC = host(gb), host(gC)
    e_b = np.abs(gb - gb0).max() / np.abs(gb0).max()
    e_C = np.abs(gC - gC0).max() / np.abs(gC0).max()
    # KKT residuals of the gradient at the point it was taken at
    G, _, _ = nt.nt_factor(Xc, Sc)
    Gi = np.linalg.inv(G)
    scale = np.linalg.norm(ops.a_op(p, G @ G.T @ GX @ G @ G.T))
    e_primal = np.linalg.norm(ops.a_op(p, gC)) / scale
    rhs = G.T @ (ops.at_op(p, gb) - GX) @ G
    e_second = np.linalg.norm(Gi @ gC @ Gi.T - rhs) / np.linalg.norm(rhs)
    print(f"tol {tol} prec {prec}: centring steps {st['centring_steps']} distance {st['centrality']:.1e} "
          f"inner its {st['inner_iterations']} e_b {e_b:.1e} e_C {e_C:.1e} primal {e_primal:.1e} second {e_second:.1e}")
    assert st["converged"] == 1 and st["centrality"] <= 1e-8
    assert e_primal <= 1e-9 and e_second <= 1e-8
    if tol >= 1e-2:
        assert e_b <= 1e-5 and e_C <= 1e-5


@pytest.mark.parametrize("n,r,seed", [(16, 2, 1), (40, 3, 2)])
@pytest.mark.parametrize("tol", [1e-2, 1e-4])
def test_adjoint_entry_sampling_matches_oracle(n, r, seed, tol):
    # entry-sampling constraints (A_i = sym(e_j e_k^T)) on a planted,
    # strictly complementary instance with m = n r - r (r - 1) / 2: both
    # problems are strictly feasible, so the central path exists and the
    # re-centring must reach it
    m = n * r - r * (r - 1) // 2
    p = workloads.planted_pair(n, r, m, seed=seed, kind="entry")
    res = ipm.solve(p, tol=tol)
    X, y, S = res["X"], res["y"], res["S"]
    GX = 2.0 * (X - target_of(n))
    gC0, gb0 = oadj.solution_gradient(p, X, y, S, GX)
    with Context(p, inner_tol=1e-13) as ctx:
        ctx.set_point(dev(X), dev(y), dev(S))
        gb, gC, st = ctx.adjoint(dev(GX))
    gb, gC = host(gb), host(gC)
    e_b = np.abs(gb - gb0).max() / np.abs(gb0).max()
    e_C = np.abs(gC - gC0).max() / np.abs(gC0).max()
    print(f"entry n {n} r {r} tol {tol}: centring steps {st['centring_steps']} distance {st['centrality']:.1e} "
          f"inner its {st['inner_iterations']} e_b {e_b:.1e} e_C {e_C:.1e}")
    assert st["status"] == L.SDP_OK and st["converged"] == 1 and st["centrality"] <= 1e-8
    assert e_b <= 1e-5 and e_C <= 1e-5


def test_adjoint_reports_missing_central_path():
    # observing 120 of the 210 entries of a rank-2 20 x 20 matrix leaves no
    # strictly feasible primal point (the oracle's centring stalls at a
    # distance ~1.6): the adjoint must say so instead of returning SDP_OK
    p = workloads.matrix_completion(20, 2, 120, seed=5)
    with Context(p) as ctx:
        ctx.solve()
        X = ctx.get_point()[0]
        G = 2.0 * (X - dev(target_of(p["n"])))
        with pytest.raises(SdpError) as ei:
            ctx.adjoint(G)
        assert ei.value.status == L.SDP_ECENTER
        _, _, st = ctx.adjoint(G, raise_off_centre=False)
    print(f"no central path: status {st['status']} distance {st['centrality']:.2e}")
    assert st["status"] == L.SDP_ECENTER and st["centrality"] > L.SDP_ADJOINT_CENTER_TOL


def test_adjoint_matches_gpu_central_path_differences():
    p = workloads.config(0)
    n, m = p["n"], p["m"]
    res = ipm.solve(p, tol=1e-2)
    target = target_of(n)

    def loss(X):
        return float(np.sum((X - target) ** 2))

    with Context(p, inner_tol=1e-13) as ctx:
        ctx.set_point(dev(res["X"]), dev(res["y"]), dev(res["S"]))
        Xs = ctx.get_point()[0]
        gb, gC, st = ctx.adjoint(2.0 * (Xs - dev(target)))  # centres first: use its point
        Xc, yc, Sc = ctx.get_point()
        gb, gC, st = ctx.adjoint(2.0 * (Xc - dev(target)))
    gb, gC = host(gb), host(gC)
    rng = np.random.default_rng(3)
    h = 1e-5
    for k in range(2):
        db = rng.standard_normal(m)
        M = rng.standard_normal((n, n))
        dC = 0.5 * (M + M.T)
        vals = []
        for sgn in (1.0, -1.0):
            with Context(oadj.perturbed(p, db, dC, sgn * h)) as cp:
                cp.set_point(Xc, yc, Sc)
                _, _, s2 = cp.adjoint(torch.zeros_like(Xc))  # moves onto the perturbed central path
                assert s2["centrality"] <= 1e-8
                vals.append(loss(host(cp.get_point()[0])))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(gb @ db + np.sum(gC * dC))
        print(f"direction {k}: adjoint {an:.8f} central-path differences {fd:.8f}")
        assert abs(an - fd) <= 1e-3 * abs(fd), (k, an, fd)


def test_layer_backward_is_the_adjoint():
    p = workloads.config(0)
    n = p["n"]
    target = dev(target_of(n))
    b = dev(p["b"]).requires_grad_(True)
    C = dev(p["C"]).requires_grad_(True)
    fixed = {"kind": "dense", "n": n, "m": p["m"], "A": p["A"]}
    opts = {"gap_tol": 1e-2, "feas_tol": 1e-2, "inner_tol": 1e-13}
    X = SDPLayer.apply(b, C, fixed, dict(opts, adjoint_inner_prec=L.SDP_PREC_F32))
    loss = ((X - target) ** 2).sum()
    loss.backward()
    # the same gradient through a context directly (FP64 inner solves)
    with Context(p, **opts) as ctx:
        ctx.solve()
        X2, _, _ = ctx.get_point()
        gb, gC, st = ctx.adjoint(2.0 * (X2 - target))
    e_b = (b.grad - gb).abs().max().item() / gb.abs().max().item()
    e_C = (C.grad - gC).abs().max().item() / gC.abs().max().item()
    print(f"layer vs context: e_b {e_b:.1e} e_C {e_C:.1e}, centring distance {st['centrality']:.1e}")
    assert torch.isfinite(b.grad).all() and torch.isfinite(C.grad).all()
    assert e_b <= 1e-4 and e_C <= 1e-4
