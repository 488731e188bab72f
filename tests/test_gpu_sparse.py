"""GPU parity of the sparse constraint kind (SDP_A_SPARSE: the entries of each A_i
on and above the diagonal), the form the SNL distance rows a a^T take at scale.

* SNL with the LP block (eq. snl-sdp): the augmented operator against the
  oracle's on the GPU's eigen-split (entry by entry) and the preconditioner
  by its backward error, at two of the oracle's iterates;
* the same SNL instance stored densely and sparsely: equal operator
  products at the same point and the same solution;
* a completion instance re-expressed as sparse entries solves like the
  entry-sampling kind;
* misuse is rejected (BF16 inner precision, the adjoint).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import certify, ipm, reform as rf  # noqa: E402
from paper_2407_14013_amd import Context, SdpError  # noqa: E402
from paper_2407_14013_amd import _lib as L  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def snl(kind):
    return workloads.sensor_localization(20, 120, 30, 3, 1, seed=2, kind=kind)


def gpu_split(ctx, n):
    g = ctx.get_scaling()
    lam, V, r = g["lam"], host(g["V"]), g["r"]
    sp = {"n": n, "r": r, "tau": 0.5 * lam[r], "lam": lam, "V": V, "Q": V[:, :r], "Qp": V[:, r:],
          "lam_top": lam[:r], "lam_perp": lam[r:]}
    return g, sp


@pytest.mark.parametrize("iters", [8, 14])
def test_sparse_snl_operator_and_precond_match_oracle(iters):
    p = snl("sparse")
    res = ipm.solve(p, maxit=iters)
    m, n = p["m"], p["n"]
    rng = np.random.default_rng(iters)
    with Context(p) as ctx:
        ctx.set_point(dev(res["X"]), dev(res["y"]), dev(res["S"]), dev(res["x"]), dev(res["s"]))
        g, sp = gpu_split(ctx, n)
        lsp = rf.lp_split(sp, host(ctx.lp_split()["w"]), cap=int(ctx.options.lp_top_max))
        beta = rf.beta_rule_lp(sp, lsp, p)
        assert abs(g["beta"] - beta) <= 1e-10 * beta, (g["beta"], beta)
        N = ctx.aug_dim()
        assert N == m + rf.dim_d(n, sp["r"]) + lsp["t"]
        E, sig = rf.e_matrix(sp), rf.sigma_diag(sp)
        errs = []
        for trial in range(3):
            x = rng.standard_normal(N)
            if trial == 1:
                x[m:] = 0.0
            if trial == 2:
                x[:m] = 0.0
            got = host(ctx.newton_apply(dev(x)))
            t, b = rf.aug_apply_lp(p, sp, lsp, E, sig, x[:m], x[m:])
            ref = np.concatenate([t, b])
            errs.append(np.abs(got - ref).max() / np.abs(ref).max())
        sig_all = np.concatenate([sig, lsp["sig"]])
        P = rf.precond_matrix(rf.aq_matrix_lp(p, sp, lsp), sp, sig_all, g["beta"])
        x = rng.standard_normal(N)
        z = host(ctx.precond_apply(dev(x)))
        bwd = np.linalg.norm(P @ z - x) / (np.linalg.norm(P, 2) * np.linalg.norm(z) + np.linalg.norm(x))
    print(f"sparse snl it {iters}: r {sp['r']} t {lsp['t']} operator errors "
          f"{', '.join(f'{e:.1e}' for e in errs)} preconditioner backward error {bwd:.1e}")
    assert max(errs) <= 1e-10 and bwd <= 1e-10


def test_dense_and_sparse_snl_agree_on_the_gpu():
    pd, ps = snl("dense"), snl("sparse")
    res = ipm.solve(pd, maxit=8)
    pts = [dev(res[k]) for k in ("X", "y", "S", "x", "s")]
    outs = []
    for p in (pd, ps):
        with Context(p) as ctx:
            ctx.set_point(*pts)
            N = ctx.aug_dim()
            xin = dev(np.random.default_rng(0).standard_normal(N))
            outs.append(host(ctx.newton_apply(xin)))
    e = np.abs(outs[0] - outs[1]).max() / np.abs(outs[0]).max()
    sols = []
    for p in (pd, ps):
        with Context(p) as ctx:
            info = ctx.solve()
            X = host(ctx.get_point()[0])
            sols.append((info, X))
    eX = np.linalg.norm(sols[0][1] - sols[1][1]) / np.linalg.norm(sols[0][1])
    d = ps["d"]
    rec = np.linalg.norm(sols[1][1][:d, d:] - ps["Ystar"])
    print(f"dense vs sparse: operator {e:.1e}; solves {sols[0][0]['iterations']} / {sols[1][0]['iterations']} its, "
          f"X difference {eX:.1e}, sparse recovery {rec:.1e}")
    assert e <= 1e-12 and eX <= 1e-8 and rec <= 1e-6


def completion_as_sparse(p):
    jk = p["jk"]
    q = dict(p)
    q["kind"] = "sparse"
    q["sp"] = {"ptr": np.arange(p["m"] + 1, dtype=np.int64), "row": jk[:, 0].astype(np.int32),
               "col": jk[:, 1].astype(np.int32), "val": np.where(jk[:, 0] == jk[:, 1], 1.0, 0.5)}
    del q["jk"]
    return q


def test_sparse_completion_solves_like_entry_kind():
    pe = workloads.matrix_completion(40, 3, 500, seed=9)
    ps = completion_as_sparse(pe)
    out = []
    for p in (pe, ps):
        with Context(p) as ctx:
            info = ctx.solve()
            X, y, S = (host(t) for t in ctx.get_point())
        c = certify.certificate(ps, X, y, S)
        out.append((info, X, c))
    eX = np.linalg.norm(out[0][1] - out[1][1]) / np.linalg.norm(out[0][1])
    rec = np.linalg.norm(out[1][1] - pe["U"] @ pe["U"].T) / np.linalg.norm(pe["U"] @ pe["U"].T)
    print(f"entry vs sparse completion: {out[0][0]['iterations']} / {out[1][0]['iterations']} its, "
          f"X difference {eX:.1e}, recovery {rec:.1e}, relgap {out[1][2]['relgap']:.1e}")
    c = out[1][2]
    assert c["pinf"] <= 1e-8 and c["dinf"] <= 1e-8 and c["relgap"] <= 1e-8
    assert eX <= 1e-7 and rec <= 1e-6


def test_sparse_kind_rejects_misuse():
    p = snl("sparse")
    with pytest.raises(SdpError) as ei:
        Context(p, inner_prec=L.SDP_PREC_BF16)
    assert ei.value.status == L.SDP_EINVAL
    q = completion_as_sparse(workloads.matrix_completion(16, 2, 100, seed=3))
    with Context(q) as ctx:
        X = ctx.get_point()[0]
        with pytest.raises(SdpError) as ei:
            ctx.adjoint(X)
        assert ei.value.status == L.SDP_EINVAL
