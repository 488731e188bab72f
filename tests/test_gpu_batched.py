"""GPU checks of the batched persistent solver (sdp_solve_batched, sdp_autotune_batched).

An uneven batch of Gaussian sensing problems (n from 18 to 30, r in {1,2,3},
m = 3 n r, the generator of the batched workload at sizes the oracle solves
in seconds), and a sample spread over the workload's whole size range (n from
16 to 128, r in {1,2,3}, including the m-capped n = 16, r = 3 case), are each
solved in one launch and every instance is checked like the
single-instance solver: objective within 1e-8 of the oracle's, relative gap
and primal infeasibility <= 1e-8 recomputed on the CPU from the returned X
and y, X positive definite and C - A^T(y) PSD to rounding, and the planted
low-rank solution recovered.  The autotuner's choice must give the same
answers, and instances solved alone must agree with the batch.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads  # noqa: E402
from oracle import ipm, operators as ops  # noqa: E402
from paper_2407_14013_amd import SdpError  # noqa: E402
from paper_2407_14013_amd import _lib as L  # noqa: E402
from paper_2407_14013_amd.batched import autotune, solve_batched  # noqa: E402


def batch(count=10, seed=7):
    return workloads.batched_sensing(count, seed=seed, n_lo=18, n_hi=30)


def check_instance(p, res, X, y, pobj_ref):
    assert res["status"] == 0, res
    X = X.detach().cpu().numpy()
    y = y.detach().cpu().numpy()
    rp = p["b"] - ops.a_op(p, X)
    pinf = np.linalg.norm(rp) / (1.0 + np.linalg.norm(p["b"]))
    pobj = float(np.sum(p["C"] * X))
    dobj = float(p["b"] @ y)
    relgap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    assert pinf <= 1.01e-8 and relgap <= 1.01e-8, (pinf, relgap)
    assert np.linalg.eigvalsh(X)[0] > 0
    S = p["C"] - ops.at_op(p, y)
    assert np.linalg.eigvalsh(S)[0] >= -1e-6 * np.linalg.norm(p["C"])
    e_obj = abs(pobj - pobj_ref) / abs(pobj_ref)
    assert e_obj <= 1e-8, (pobj, pobj_ref)
    Xs = p["U"] @ p["U"].T
    return e_obj, np.linalg.norm(X - Xs) / np.linalg.norm(Xs)


PRECS = [L.SDP_PREC_F64, L.SDP_PREC_F32]


@pytest.mark.parametrize("prec", PRECS)
def test_batched_matches_oracle(prec):
    # prec F32: the inner operator over FP32 rows with E Y E on the FP32
    # matrix cores, FP64 refinement of every Newton step -- the same bars
    probs = batch()
    refs = [ipm.solve(p)["history"][-1]["pobj"] for p in probs]
    results, Xs, ys = solve_batched(probs, want_y=True, inner_prec=prec)
    for i, p in enumerate(probs):
        e_obj, e_rec = check_instance(p, results[i], Xs[i], ys[i], refs[i])
        r = results[i]
        print(f"instance {i} prec {prec}: n {p['n']} r {p['r']} m {p['m']} its {r['iterations']} "
              f"pcg {r['pcg_iterations']} products fp64 {r['newton_matvecs']} low {r['lp_matvecs']} "
              f"objective error {e_obj:.1e} recovery {e_rec:.1e}")
        assert e_rec <= 1e-6
        assert (r["lp_matvecs"] > 0) == (prec == L.SDP_PREC_F32)


def test_batched_autotune_and_single_instances_agree():
    probs = batch(count=6, seed=8)
    tune, ms = autotune(probs)
    assert all(t.rows_per_wave in (1, 2, 4) and t.aq_group in (4, 8, 16) and t.gemm_tile in (16, 32) for t in tune)
    r_all, X_all, _ = solve_batched(probs, tune=tune)
    for i, p in enumerate(probs):
        r_one, X_one, _ = solve_batched([p])
        assert r_all[i]["status"] == 0 and r_one[0]["status"] == 0
        e = abs(r_all[i]["pobj"] - r_one[0]["pobj"]) / abs(r_one[0]["pobj"])
        assert e <= 1e-10


# (n, r) across the batched workload's range: n = 16 with r = 3 has m = 3 n r
# = 144 capped at n (n + 1) / 2 = 136, the largest instances have n = 128
SPREAD = [(16, 3), (40, 1), (64, 2), (96, 3), (128, 1), (128, 3)]


@pytest.fixture(scope="module")
def spread():
    probs = [workloads.gaussian_sensing(n, r, min(3 * n * r, n * (n + 1) // 2), seed=100 + i)
             for i, (n, r) in enumerate(SPREAD)]
    assert probs[0]["m"] == 136
    return probs, [ipm.solve(p)["history"][-1]["pobj"] for p in probs]


@pytest.mark.parametrize("prec", PRECS)
def test_batched_size_spread_matches_oracle(spread, prec):
    probs, refs = spread
    results, Xs, ys = solve_batched(probs, want_y=True, inner_prec=prec)
    for i, p in enumerate(probs):
        e_obj, e_rec = check_instance(p, results[i], Xs[i], ys[i], refs[i])
        r = results[i]
        print(f"instance {i} prec {prec}: n {p['n']} r {p['r']} m {p['m']} its {r['iterations']} "
              f"pcg {r['pcg_iterations']} products fp64 {r['newton_matvecs']} low {r['lp_matvecs']} "
              f"objective error {e_obj:.1e} recovery {e_rec:.1e}")
        assert e_rec <= 1e-6


@pytest.mark.parametrize("prec", PRECS)
def test_batched_16_wide_wave_tiles_match_oracle(spread, prec):
    # the workgroup's MFMA products with 16 x 16 wave tiles (gemm_tile 16)
    probs, refs = spread
    tune = (L.SdpBatchTune * len(probs))(*[L.SdpBatchTune(2, 8, 16) for _ in probs])
    results, Xs, ys = solve_batched(probs, tune=tune, want_y=True, inner_prec=prec)
    for i, p in enumerate(probs):
        e_obj, e_rec = check_instance(p, results[i], Xs[i], ys[i], refs[i])
        assert e_rec <= 1e-6, (i, e_obj, e_rec)


def test_batched_rejects_bf16_inner():
    with pytest.raises(SdpError):
        solve_batched(batch(count=2), inner_prec=L.SDP_PREC_BF16)
