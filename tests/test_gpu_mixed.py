"""GPU checks of the mixed-precision mode (FP32 / BF16 inner operator + FP64 refinement).

* wc_gemm_lp: FP32 and BF16 matrix-core GEMMs with FP32 accumulation against
  the exact FP64 product of the same rounded operands.  Bound: a length-K
  FP32 sum, |error| <= 2 K u32 sum_k |a_ik||b_kj| (u32 = 2^-24), plus one
  output rounding (u32, or u_bf16 = 2^-8 for BF16 output).
* wc_to_lowp: BF16 rounding is bit-exact against round-to-nearest-even of the
  FP32 value.
* sdp_newton_apply_prec: the low-precision operator against the oracle's
  FP64 products (Section 5); the difference is the rounding of the data and
  of the GEMM operands, bounded relative to the largest output entry.
* sdp_inner_solve / sdp_solve in FP32 and BF16 modes: the same residual bars
  and objective tolerance as the FP64 mode -- the refinement restores FP64
  accuracy of the Newton step -- plus the error against the FP64 oracle
  stated per result.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import certify, ipm, nt, operators as ops, reform as rf  # noqa: E402
from paper_2407_14013_amd import Context  # noqa: E402
from paper_2407_14013_amd import _lib as L  # noqa: E402
from paper_2407_14013_amd import linalg as la  # noqa: E402

GOLDEN1 = os.path.join(os.path.dirname(__file__), "golden", "oracle_config1.json")
U32 = 2.0 ** -24
UBF = 2.0 ** -8
PRECS = [L.SDP_PREC_F32, L.SDP_PREC_BF16]


def bf16_bits(x):
    """Round-to-nearest-even of the FP32 value to BF16, as 16-bit patterns."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rounded(A, prec):
    """(device low-precision copy, exact FP64 value of it) of a numpy matrix."""
    lp = la.to_lowp(la.to_dev(A), prec)
    if prec == L.SDP_PREC_F32:
        val = host(lp).T.astype(np.float64)
    else:
        val = bf16_value(host(lp).view(np.uint16).T)
    return lp, val


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (17, 33, 9), (64, 64, 64), (130, 67, 95), (200, 200, 200), (65, 3, 257)])
def test_gemm_lp(prec, m, n, k):
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    Al, Av = rounded(A, prec)
    Bl, Bv = rounded(B, prec)
    exact = Av @ Bv
    mag = np.abs(Av) @ np.abs(Bv)
    # FP32 output
    got = host(la.gemm_lp(prec, 0, Al, Bl)).T.astype(np.float64)
    e = np.abs(got - exact) - (2 * k * U32 * mag + U32 * np.abs(exact))
    assert e.max() <= 0
    # BF16 output
    got = bf16_value(host(la.gemm_lp(prec, 1, Al, Bl)).view(np.uint16).T)
    e = np.abs(got - exact) - (2 * k * U32 * mag * (1 + UBF) + UBF * np.abs(exact))
    assert e.max() <= 0
    # FP64 output
    got = la.from_dev(la.gemm_lp(prec, 3, Al, Bl, la.to_dev(np.full((m, n), np.nan))))
    e = np.abs(got - exact) - (2 * k * U32 * mag + U32 * np.abs(exact))
    assert e.max() <= 0
    # FP64 accumulate: C0 + A B
    C0 = rng.standard_normal((m, n))
    Cd = la.to_dev(C0)
    la.gemm_lp(prec, 2, Al, Bl, Cd)
    got = la.from_dev(Cd)
    e = np.abs(got - (C0 + exact)) - (2 * k * U32 * mag + U32 * np.abs(exact))
    assert e.max() <= 0


@pytest.mark.parametrize("prec,m,n", [(p, m, n) for p in PRECS
                                       for m, n in [(17, 5), (200, 200), (1032, 1032), (1100, 1030), (2056, 520)]]
                         + [(L.SDP_PREC_BF16, 4000, 4000), (L.SDP_PREC_BF16, 3896, 3620)])
def test_gemm_lp_sym(prec, m, n):
    # the product with a symmetric left operand (the E Y E products of the
    # operator), same bounds as test_gemm_lp with K = m; m = 17 (rows not
    # 16-byte aligned) and m = 200 (fewer than 64 tiles) take the general
    # kernel, the others the 128 x 128 tiles with ragged row, column and K
    # edges; in BF16 at m = 4000 and m = 3896 (ragged edges and K, 240 and 256
    # tiles) the 256 x 256-tile kernel
    rng = np.random.default_rng(m * 5 + n)
    M0 = rng.standard_normal((m, m))
    A = 0.5 * (M0 + M0.T)
    B = rng.standard_normal((m, n))
    Al, Av = rounded(A, prec)
    Bl, Bv = rounded(B, prec)
    exact = Av @ Bv
    mag = np.abs(Av) @ np.abs(Bv)
    got = host(la.gemm_lp_sym(prec, 0, Al, Bl)).T.astype(np.float64)
    assert (np.abs(got - exact) - (2 * m * U32 * mag + U32 * np.abs(exact))).max() <= 0
    got = bf16_value(host(la.gemm_lp_sym(prec, 1, Al, Bl)).view(np.uint16).T)
    assert (np.abs(got - exact) - (2 * m * U32 * mag * (1 + UBF) + UBF * np.abs(exact))).max() <= 0
    got = la.from_dev(la.gemm_lp_sym(prec, 3, Al, Bl, la.to_dev(np.full((m, n), np.nan))))
    assert (np.abs(got - exact) - (2 * m * U32 * mag + U32 * np.abs(exact))).max() <= 0
    C0 = rng.standard_normal((m, n))
    Cd = la.to_dev(C0)
    la.gemm_lp_sym(prec, 2, Al, Bl, Cd)
    got = la.from_dev(Cd)
    assert (np.abs(got - (C0 + exact)) - (2 * m * U32 * mag + U32 * np.abs(exact))).max() <= 0


def test_to_lowp_bf16_is_round_to_nearest_even():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((37, 29)) * np.exp(rng.uniform(-30, 30, (37, 29)))
    A[0, :4] = [0.0, -0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8]  # exact ties go to even
    got = host(la.to_lowp(la.to_dev(A), L.SDP_PREC_BF16)).view(np.uint16).T
    assert np.array_equal(got, bf16_bits(A.astype(np.float32)))
    got32 = host(la.to_lowp(la.to_dev(A), L.SDP_PREC_F32)).T
    assert np.array_equal(got32, A.astype(np.float32))


def small_entry():
    return workloads.matrix_completion(16, 2, 100, seed=3)


def ipm_point(p, iters):
    res = ipm.solve(p, maxit=iters)
    return res["X"], res["y"], res["S"]


# Bound on the low-precision operator's error relative to the largest output
# entry: FP32 -- rounding of the packed rows and of E, Y (u32 each) amplified
# by the cancellation in the length-N2 sums (~sqrt(N2)); BF16 -- the GEMM
# operands' u_bf16 = 2^-8, likewise amplified.
LP_TOL = {L.SDP_PREC_F32: 2e-5, L.SDP_PREC_BF16: 5e-2}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("which", ["cfg0", "entry", "cfg1"])
def test_newton_apply_lowp_close_to_oracle(prec, which):
    p = {"cfg0": lambda: workloads.config(0), "entry": small_entry, "cfg1": lambda: workloads.config(1)}[which]()
    m = p["m"]
    if which == "cfg1":
        X, S = workloads.random_pd_pair(p["n"], seed=5, spread=1.0)
        y = np.zeros(m)
    else:
        X, y, S = ipm_point(p, 4)
    with Context(p, inner_prec=prec) as ctx:
        ctx.set_point(dev(X), dev(y), dev(S))
        N = ctx.aug_dim()
        x = np.random.default_rng(2).standard_normal(N)
        got = host(ctx.newton_apply(dev(x), prec=prec))
        got64 = host(ctx.newton_apply(dev(x)))
    G, d, Lf = nt.nt_factor(X, S)
    sp = rf.eig_split(G @ G.T)
    t, b = rf.aug_apply(p, sp, rf.e_matrix(sp), rf.sigma_diag(sp), x[:m], x[m:])
    ref = np.concatenate([t, b])
    e64 = np.abs(got64 - ref).max() / np.abs(ref).max()
    elp = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"{which} prec {prec}: fp64 err {e64:.2e}, low-precision err {elp:.2e}")
    assert e64 <= 1e-10
    assert elp <= LP_TOL[prec]
    assert elp > 0  # the low-precision path really ran


MODES = [L.SDP_REFINE_SWEEPS, L.SDP_REFINE_REPLACE]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("which", ["cfg0", "entry", "entry_sampled"])
@pytest.mark.parametrize("iters", [2, 6])
def test_inner_solve_mixed_meets_fp64_bars(prec, which, iters, mode):
    # both refinement modes (restarted sweeps, FP64 residual replacement);
    # entry_sampled takes the FP64 residuals with the sampled A(E Y E)
    p = workloads.config(0) if which == "cfg0" else small_entry()
    X, y, S = ipm_point(p, iters)
    r = ipm.residuals(p, X, y, S)
    Ct = r["Rd"] + S
    bt = r["rp"]
    G, d, Lf = nt.nt_factor(X, S)
    W = G @ G.T
    with Context(p, inner_prec=prec, refine_mode=mode, sparse_sandwich=int(which == "entry_sampled")) as ctx:
        ctx.set_point(dev(X), dev(y), dev(S))
        dX, dy, st = ctx.inner_solve(dev(bt), dev(Ct))
    dX, dy = host(dX), host(dy)
    assert st["converged"] == 1 and st["rel_res"] <= 1e-10 and st["refinements"] >= 1
    scale = np.linalg.norm(bt + ops.a_op(p, W @ Ct @ W))
    e_primal = np.linalg.norm(ops.a_op(p, dX) - bt) / scale
    Gi = np.linalg.inv(G)
    rhs = G.T @ (ops.at_op(p, dy) - Ct) @ G
    e_second = np.linalg.norm(Gi @ dX @ Gi.T - rhs) / np.linalg.norm(rhs)
    print(f"{which} it {iters} prec {prec} mode {mode}: sweeps {st['refinements']} pcg {st['iterations']} "
          f"primal {e_primal:.1e} second {e_second:.1e}")
    assert e_primal <= 1e-9
    assert e_second <= 1e-8


def _solve(p, prec, **kw):
    with Context(p, inner_prec=prec, **kw) as ctx:
        res = ctx.solve()
        X, y, S = ctx.get_point()
    return res, host(X), host(y), host(S)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", PRECS)
def test_solve_mixed_config0_and_entry(prec, mode):
    for p in (workloads.config(0), small_entry()):
        ref = ipm.solve(p)
        res, X, y, S = _solve(p, prec, refine_mode=mode)
        assert res["status"] == 0 and res["lp_matvecs"] > 0
        c = certify.certificate(p, X, y, S)
        assert c["pinf"] <= 1.01e-8 and c["dinf"] <= 1.01e-8 and c["relgap"] <= 1.01e-8, c
        e_obj = abs(c["pobj"] - ref["history"][-1]["pobj"]) / abs(ref["history"][-1]["pobj"])
        e_X = np.linalg.norm(X - ref["X"]) / np.linalg.norm(ref["X"])
        print(f"n={p['n']} prec {prec}: objective error {e_obj:.1e}, ||X - X_oracle|| / ||X_oracle|| {e_X:.1e}")
        assert e_obj <= 1e-8
        assert e_X <= 1e-6


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", PRECS)
def test_solve_mixed_config1_matches_oracle(prec, mode):
    with open(GOLDEN1) as f:
        gold = json.load(f)
    p = workloads.config(1)
    res, X, y, S = _solve(p, prec, refine_mode=mode)
    assert res["status"] == 0 and res["lp_matvecs"] > 0
    c = certify.certificate(p, X, y, S)
    assert c["pinf"] <= 1.01e-8 and c["dinf"] <= 1.01e-8 and c["relgap"] <= 1.01e-8, c
    e_obj = abs(c["pobj"] - gold["certificate"]["pobj"]) / abs(gold["certificate"]["pobj"])
    Xs = p["U"] @ p["U"].T
    e_rec = np.linalg.norm(X - Xs) / np.linalg.norm(Xs)
    print(f"n=200 sensing, prec {prec} mode {mode}: objective error {e_obj:.1e}, planted recovery {e_rec:.1e}, "
          f"fp64 matvecs {res['newton_matvecs']}, low-precision matvecs {res['lp_matvecs']}")
    assert e_obj <= 1e-8
    assert e_rec <= 1e-6
