"""Benchmark: Newton-operator mat-vecs per second and IPM time to a 1e-8 gap.

One step = one full FP64 interior-point solve (sdp_solve) of the dense
Gaussian matrix-sensing workload n=200, r=3, m=2400 from the standard
starting point to relative gap, primal and dual infeasibility <= 1e-8.  The
constraint data is resident in HBM before timing starts (the setup upload
and packing are outside the timed region).  value = augmented-operator
applications performed by the timed solves / timed seconds.

The JSON line also carries:
  roofline      the dominant kernel (the packed A / A^T passes, HBM bound)
                timed live with HIP events on the library's stream;
  cpu_baseline  the CPU oracle's augmented operator on the same workload
                (bounded sample, all host cores);
  newton_apply  a tight loop of sdp_newton_apply at the final scaling point.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "packed_passes_gaussian_n200_m2400_hbm_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2407_14013_amd", "csrc", "blas.hip")
METRIC = "Newton-op matvecs/s and IPM time-to-1e-8 gap, FP64 vs mixed prec, 1 GPU"
WORKLOAD = "gaussian sensing SDP n=200 r=3 m=2400 (dense A, FP64)"


def cpu_baseline(p, budget_s=15.0):
    """The oracle's Section 5 operator timed on the host cores."""
    from oracle import nt, reform as rf

    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    X, S = __import__("workloads").random_pd_pair(p["n"], seed=5, spread=1.0)
    G, d, L = nt.nt_factor(X, S)
    sp = rf.eig_split(G @ G.T)
    E = rf.e_matrix(sp)
    sig = rf.sigma_diag(sp)
    m = p["m"]
    N = m + rf.dim_d(p["n"], sp["r"])
    x = np.random.default_rng(0).standard_normal(N)
    rf.aug_apply(p, sp, E, sig, x[:m], x[m:])
    calls = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        rf.aug_apply(p, sp, E, sig, x[:m], x[m:])
        calls += 1
    el = time.perf_counter() - t0
    return {
        "value": calls / el,
        "unit": "matvec/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{calls} applications of the oracle's augmented operator (eq. augsys via the Section 5 products) "
                  f"on the same workload at a fixed scaling point, {el:.1f} s",
    }


def packed_source_digest():
    """SHA-256 of the source text of the two packed-pass kernels and their launchers."""
    import hashlib

    src = open(KERNEL_SOURCE).read()
    a = src.index("constexpr int PK_ROWS")
    b = src.index("void packed_cols_partial(")
    b = src.index("\n}\n", b) + 3
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter runs.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each divided by what the
    same counter read per byte for a device copy of known size in the same run.
    None when no record exists or the kernel source changed since it was taken.
    """
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != packed_source_digest() or kernel not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][kernel]
    return 1024.0 * (k["fetch_kib"] / rec["copy"]["fetch_factor"] + k["write_kib"] / rec["copy"]["write_factor"])


def pmc_pass():
    """Short run for the rocprofv3 counter passes: operator applications plus a copy of known size."""
    import torch

    import workloads
    from paper_2407_14013_amd import Context

    torch.cuda.set_device(0)
    ctx = Context(workloads.config(1))
    N = ctx.aug_dim()
    xin = torch.randn(N, dtype=torch.float64, device="cuda")
    xout = torch.empty_like(xin)
    for _ in range(10):
        ctx.newton_apply(xin, xout)
    src = torch.randn(64 << 20, dtype=torch.float64, device="cuda")  # 512 MiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(f"pmc pass: 10 operator applications, 3 copies of {src.numel() * 8} bytes", flush=True)


def bench_batched(args):
    """The batched workload: 1024 Gaussian sensing SDPs (n in [16,128], r in {1,2,3}, m = 3nr) in one persistent launch."""
    import torch

    import workloads
    from paper_2407_14013_amd.batched import autotune, solve_batched

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    probs = workloads.config(3)
    gen_s = time.perf_counter() - t0
    print(f"generated {len(probs)} instances in {gen_s:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tune, bucket_ms = autotune(probs)
    tune_s = time.perf_counter() - t0
    print(f"autotuned in {tune_s:.1f} s", file=sys.stderr, flush=True)
    results, Xs, _ = solve_batched(probs, tune=tune)
    torch.cuda.synchronize()
    launch_ms = results[0]["time_ms"]
    ok = sum(r["status"] == 0 for r in results)
    # algorithmic bytes of the packed constraint passes: two passes per PCG iteration
    nbytes = 0.0
    for p, r in zip(probs, results):
        ldp = (p["n"] * (p["n"] + 1) // 2 + 1) // 2 * 2
        nbytes += 2.0 * r["pcg_iterations"] * p["m"] * ldp * 8
    line = {
        "metric": "IPM time-to-1e-8 gap, batched",
        "value": len(probs) / (launch_ms * 1e-3),
        "unit": "instances/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1024 gaussian sensing SDPs, n in [16,128], r in {1,2,3}, m = 3nr (dense A, FP64)"},
        "launch_ms": launch_ms,
        "solved": ok,
        "ipm_iterations_total": int(sum(r["iterations"] for r in results)),
        "pcg_iterations_total": int(sum(r["pcg_iterations"] for r in results)),
        "autotune": {"bucket_ms": bucket_ms, "configs": sorted({(t.rows_per_wave, t.aq_group) for t in tune})},
        "a_pass_bytes": nbytes,
        "a_pass_gbs_lower_bound": nbytes / (launch_ms * 1e-3) / 1e9,
        "generate_s": gen_s,
    }
    if not args.no_cpu_baseline:
        from oracle import ipm

        try:
            from threadpoolctl import threadpool_info

            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        sample = sorted(range(len(probs)), key=lambda i: probs[i]["m"] * probs[i]["n"] ** 2)[::128][:6]
        t0 = time.perf_counter()
        for i in sample:
            ipm.solve(probs[i])
        el = time.perf_counter() - t0
        work = sum(probs[i]["m"] * probs[i]["n"] ** 2 for i in sample)
        total = sum(p["m"] * p["n"] ** 2 for p in probs)
        line["cpu_baseline"] = {
            "value": len(probs) / (el * total / work),
            "unit": "instances/s",
            "cores": int(threads),
            "kind": "oracle",
            "sample": f"{len(sample)} instances spread over the size range solved by the oracle in {el:.1f} s, "
                      f"scaled to the whole batch by sum(m n^2)",
        }
    print(json.dumps(line))


def bench_adjoint(args):
    """The adjoint workload: FP64 solve of the n=1000 completion SDP, then the KKT adjoint with the FP32 inner operator."""
    import torch

    import workloads
    from paper_2407_14013_amd import Context
    from paper_2407_14013_amd import _lib as L

    torch.cuda.set_device(0)
    p = workloads.config(4)
    n = p["n"]
    V = np.random.default_rng(1).standard_normal((n, 3))
    target = torch.from_numpy(V @ V.T).cuda()
    with Context(p) as fwd:
        t0 = time.perf_counter()
        res = fwd.solve()
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        X, y, S = fwd.get_point()
    with Context(p, inner_prec=L.SDP_PREC_F32) as bwd:
        bwd.set_point(X, y, S)
        t0 = time.perf_counter()
        gb, gC, st = bwd.adjoint(2.0 * (X - target), raise_off_centre=False)
        torch.cuda.synchronize()
        t_bwd = time.perf_counter() - t0
    line = {
        "metric": "SDP layer forward (FP64 solve) and backward (FP32-inner KKT adjoint) time",
        "value": t_fwd + t_bwd,
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "matrix completion SDP n=1000 r=3 m=30000, loss ||X - X_target||_F^2"},
        "forward": {"time_s": t_fwd, "iterations": res["iterations"], "pcg_iterations": res["pcg_iterations"],
                    "relgap": res["relgap"]},
        "backward": {"time_s": t_bwd, "status": L.STATUS_NAMES.get(st.pop("status")), **st},
        "grad_norms": {"dL_db": float(gb.norm()), "dL_dC": float(gC.norm())},
    }
    print(json.dumps(line))


MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}


def bench_completion(args):
    """The n=4000 matrix-completion operator, where E Y E on the matrix cores dominates.

    At a closed-form centred point with a rank-4 split (the shape of the late
    iterates) every form of the operator is applied in a tight loop: FP64,
    and the FP32 and BF16 forms that the refinement sweeps use.  The two
    n x n x n GEMMs of E Y E are timed by the library with HIP events on its
    stream (kernel class SDP_K_SANDWICH): 2 n^3 flops per launch.  With
    --solve, the full solves to the 1e-8 tolerances are timed as well
    (minutes): FP64 with the sampled A(E Y E) form, FP64 with the dense
    products, FP32-mixed and BF16-mixed.  The sampled form (sparse_sandwich) is timed
    per kernel class too: Z = Y E and the per-constraint dot products.
    """
    import torch

    import workloads
    from paper_2407_14013_amd import Context
    from paper_2407_14013_amd import _lib as L

    torch.cuda.set_device(0)
    p = workloads.config(2)
    n, m, r0, mu = p["n"], p["m"], 4, 1e-2
    X, S, V, x, s = workloads.centred_pair(n, r0, mu, seed=21)
    Xd, Sd = torch.from_numpy(X).cuda(), torch.from_numpy(S).cuda()
    yd = torch.zeros(m, dtype=torch.float64, device="cuda")
    del X, S
    flops = 2.0 * n ** 3
    forms = {}
    wanted_forms = args.forms.split(",")
    for name, prec, sparse in (("f64", L.SDP_PREC_F64, 0), ("f32", L.SDP_PREC_F32, 0), ("bf16", L.SDP_PREC_BF16, 0),
                               ("f64_sampled", L.SDP_PREC_F64, 1)):
        if name not in wanted_forms:
            continue
        with Context(p, inner_prec=prec, sparse_sandwich=sparse) as ctx:
            ctx.set_point(Xd, yd, Sd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sc = ctx.get_scaling()
            torch.cuda.synchronize()
            t_scaling = time.perf_counter() - t0
            N = ctx.aug_dim()
            xin = torch.randn(N, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
            xout = torch.empty_like(xin)
            pr = None if prec == L.SDP_PREC_F64 else prec
            for _ in range(3):
                ctx.newton_apply(xin, xout, prec=pr)
            torch.cuda.synchronize()
            classes = [L.SDP_K_SAMPLED_YE, L.SDP_K_SAMPLED_DOTS] if sparse else [L.SDP_K_SANDWICH]
            ctx.profile_enable(classes)
            calls = args.apply_loop
            t0 = time.perf_counter()
            for _ in range(calls):
                ctx.newton_apply(xin, xout, prec=pr)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            prof = {k: ctx.profile_get(k) for k in classes}
            ctx.profile_enable([])
            t0 = time.perf_counter()
            for _ in range(20):
                ctx.precond_apply(xin, xout)
            torch.cuda.synchronize()
            t_prec = (time.perf_counter() - t0) / 20
            forms[name] = {
                "matvec_per_s": calls / el,
                "ms_per_matvec": 1e3 * el / calls,
                "precond_apply_ms": 1e3 * t_prec,
                "scaling_setup_s": t_scaling,
                "r": sc["r"],
                "d": N - m,
            }
            if sparse:
                # the two sampled kernels, HBM-bound: algorithmic bytes per launch
                # as the library counts them (one column of Z per constraint)
                for key, k in (("sampled_ye", L.SDP_K_SAMPLED_YE), ("sampled_dots", L.SDP_K_SAMPLED_DOTS)):
                    pk = prof[k]
                    gbs = pk["bytes"] / (pk["ms"] * 1e-3) / 1e9
                    forms[name][key] = {"launches": pk["launches"], "avg_launch_ms": pk["ms"] / pk["launches"],
                                        "bytes_per_launch": pk["bytes"] / pk["launches"], "achieved_gbs": gbs,
                                        "peak_gbs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS}
                note = (f"Y E {forms[name]['sampled_ye']['avg_launch_ms']:.3f} ms, dots "
                        f"{forms[name]['sampled_dots']['avg_launch_ms']:.3f} ms")
            else:
                sw = prof[L.SDP_K_SANDWICH]
                tf = flops * sw["launches"] / (sw["ms"] * 1e-3) / 1e12
                forms[name]["sandwich_gemm"] = {"launches": sw["launches"], "avg_launch_ms": sw["ms"] / sw["launches"],
                                                "achieved_tflops": tf, "peak_tflops": MFMA_PEAK_TFLOPS[name],
                                                "frac": tf / MFMA_PEAK_TFLOPS[name]}
                note = f"sandwich GEMM {tf:.1f} TFLOP/s"
        print(f"{name}: {forms[name]['ms_per_matvec']:.3f} ms per operator product, {note}, "
              f"scaling setup {t_scaling:.2f} s", file=sys.stderr, flush=True)
    # the line's value and roofline: the FP64 dense-product form when it was
    # run, else the FP64 sampled form with its per-constraint dot kernel
    head = "f64" if "f64" in forms else "f64_sampled"
    f64 = forms[head]
    if head == "f64":
        roof = {
            "kernel": "dgemm_kernel<false, false>: the two n x n x n products of E Y E",
            "bound": "mfma",
            "achieved": f64["sandwich_gemm"]["achieved_tflops"],
            "peak": MFMA_PEAK_TFLOPS["f64"],
            "unit": "TFLOP/s",
            "frac": f64["sandwich_gemm"]["frac"],
            "traffic": None,
            "flops_per_launch": flops,
            "avg_launch_ms": f64["sandwich_gemm"]["avg_launch_ms"],
        }
    else:
        dots = f64["sampled_dots"]
        roof = {
            "kernel": "sampled_dots_kernel: E[:, j] . Z[:, k] per constraint",
            "bound": "hbm",
            "achieved": dots["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dots["frac"],
            "traffic": None,
            "bytes_per_launch": dots["bytes_per_launch"],
            "avg_launch_ms": dots["avg_launch_ms"],
        }
    line = {
        "metric": METRIC,
        "value": f64["matvec_per_s"],
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.apply_loop,
        "warmup": 3,
        "ms_per_step": f64["ms_per_matvec"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "matrix completion SDP n=4000 r=4 m=160000 (entry sampling) at a centred point, "
                               "mu=1e-2, rank-4 split", "form": head},
        "forms": forms,
        "roofline": roof,
    }
    if args.solve:
        solves = {}
        wanted = args.solve.split(",")
        for name, prec, sparse in (("f64_sampled", L.SDP_PREC_F64, 1), ("f64", L.SDP_PREC_F64, 0),
                                   ("f32", L.SDP_PREC_F32, 0), ("bf16", L.SDP_PREC_BF16, 0)):
            if name not in wanted:
                continue
            with Context(p, inner_prec=prec, sparse_sandwich=sparse, verbose=1 if args.verbose else 0) as ctx:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = ctx.solve(raise_on_stall=False)
                torch.cuda.synchronize()
                solves[name] = {"time_to_gap_s": time.perf_counter() - t0, "status": res["status"],
                                "iterations": res["iterations"], "pcg_iterations": res["pcg_iterations"],
                                "fp64_matvecs": res["newton_matvecs"], "lowp_matvecs": res["lp_matvecs"],
                                "relgap": res["relgap"], "pinf": res["pinf"], "dinf": res["dinf"],
                                "pobj": res["pobj"]}
            print(f"solve {name}: {solves[name]}", file=sys.stderr, flush=True)
        line["ipm"] = solves
    if not args.no_cpu_baseline:
        from oracle import reform as rf

        try:
            from threadpoolctl import threadpool_info

            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        w = np.sqrt(x / s)
        order = np.argsort(-w, kind="stable")
        lam, Vo = w[order], V[:, order]
        sp = {"n": n, "r": r0, "tau": 0.5 * lam[r0], "lam": lam, "V": Vo, "Q": Vo[:, :r0], "Qp": Vo[:, r0:],
              "lam_top": lam[:r0], "lam_perp": lam[r0:]}
        E = rf.e_matrix(sp)
        sig = rf.sigma_diag(sp)
        xh = np.random.default_rng(0).standard_normal(m + rf.dim_d(n, r0))
        calls = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 15.0:
            rf.aug_apply(p, sp, E, sig, xh[:m], xh[m:])
            calls += 1
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {
            "value": calls / el,
            "unit": "matvec/s",
            "cores": int(threads),
            "kind": "oracle",
            "sample": f"{calls} applications of the oracle's augmented operator (Section 5 products) on the same "
                      f"workload and point, split supplied in closed form, {el:.1f} s",
        }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--apply-loop", type=int, default=200)
    ap.add_argument("--pmc-pass", action="store_true", help="only the short run profiled for HBM counters")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision solves")
    ap.add_argument("--workload", choices=["sensing", "batched", "adjoint", "completion"], default="sensing",
                    help="sensing: the headline line (n=200 dense); batched: 1024 small SDPs in one launch; "
                         "adjoint: n=1000 completion forward + backward; completion: n=4000 completion operator")
    ap.add_argument("--verbose", action="store_true",
                    help="completion --solve: one line per interior-point iteration on stderr")
    ap.add_argument("--forms", default="f64,f32,bf16,f64_sampled",
                    help="completion: operator forms to time (comma list of f64, f32, bf16, f64_sampled)")
    ap.add_argument("--solve", nargs="?", const="f64_sampled,f64,f32,bf16", default="",
                    help="completion: also time full solves, a comma list of f64_sampled, f64, f32, bf16 "
                         "(default all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every instance of this workload fits one MI355X, "
              "and the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.pmc_pass:
        pmc_pass()
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "adjoint":
        bench_adjoint(args)
        return
    if args.workload == "completion":
        bench_completion(args)
        return

    import torch

    import workloads
    from paper_2407_14013_amd import Context
    from paper_2407_14013_amd import _lib as L

    torch.cuda.set_device(0)
    p = workloads.config(1)
    ctx = Context(p)
    X0, y0, S0 = (t.clone() for t in ctx.get_point())

    def one_solve():
        ctx.set_point(X0, y0, S0)
        return ctx.solve()

    for _ in range(args.warmup):
        one_solve()
    torch.cuda.synchronize()
    ctx.profile_enable([L.SDP_K_A_APPLY, L.SDP_K_AT_APPLY])
    results = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(one_solve())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {k: ctx.profile_get(k) for k in (L.SDP_K_A_APPLY, L.SDP_K_AT_APPLY, L.SDP_K_GEMM, L.SDP_K_NEWTON)}
    ctx.profile_enable([])
    matvecs = sum(r["newton_matvecs"] for r in results)
    for r in results:
        assert r["status"] == 0 and r["relgap"] <= 1e-8, r

    # one more FP64 solve step by step (untimed): mu, rank and PCG iterations of
    # the predictor and corrector systems along the trajectory (Corollary pcg:
    # the counts stay bounded as mu -> 0)
    ctx.set_point(X0, y0, S0)
    trajectory = []
    for _ in range(100):
        st = ctx.ipm_step()
        if st["converged"]:
            break
        trajectory.append({"mu": st["mu"], "relgap": st["relgap"], "r": st["r"], "pcg_pred": st["pcg_pred"],
                           "pcg_corr": st["pcg_corr"]})

    # the same solves with the mixed-precision inner operator
    mixed = {}
    if not args.no_mixed:
        for name, prec in (("f32", L.SDP_PREC_F32), ("bf16", L.SDP_PREC_BF16)):
            mctx = Context(p, inner_prec=prec)
            mctx.set_point(X0, y0, S0)

            def msolve():
                mctx.set_point(X0, y0, S0)
                return mctx.solve()

            for _ in range(args.warmup):
                msolve()
            torch.cuda.synchronize()
            mres = []
            tm0 = time.perf_counter()
            for _ in range(args.steps):
                mres.append(msolve())
            torch.cuda.synchronize()
            mel = time.perf_counter() - tm0
            mctx.close()
            for r in mres:
                assert r["status"] == 0 and r["relgap"] <= 1e-8, r
            mixed[name] = {
                "time_to_gap_s": mel / args.steps,
                "speedup_vs_fp64": (el / args.steps) / (mel / args.steps),
                "iterations": mres[-1]["iterations"],
                "fp64_matvecs": mres[-1]["newton_matvecs"],
                "lowp_matvecs": mres[-1]["lp_matvecs"],
                "relgap": mres[-1]["relgap"],
                "pobj_rel_diff_vs_fp64": abs(mres[-1]["pobj"] - results[-1]["pobj"]) / abs(results[-1]["pobj"]),
            }

    # dominant kernel: the larger total time of the two packed passes over A
    kcls = max((L.SDP_K_A_APPLY, L.SDP_K_AT_APPLY), key=lambda k: prof[k]["ms"])
    kp = prof[kcls]
    avg_ms = kp["ms"] / max(kp["launches"], 1)
    bytes_per = kp["bytes"] / max(kp["launches"], 1)
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9
    kname = "packed_rows_kernel" if kcls == L.SDP_K_A_APPLY else "packed_cols_partial_kernel"
    traffic = measured_traffic(kname)

    # tight loop of the operator at the final point
    N = ctx.aug_dim()
    xin = torch.randn(N, dtype=torch.float64, device="cuda")
    xout = torch.empty_like(xin)
    for _ in range(5):
        ctx.newton_apply(xin, xout)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.apply_loop):
        ctx.newton_apply(xin, xout)
    torch.cuda.synchronize()
    loop_rate = args.apply_loop / (time.perf_counter() - t1)

    line = {
        "metric": METRIC,
        "value": matvecs / el,
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "precision": "fp64", "ipm_tol": 1e-8, "inner_tol": 1e-10},
        "ipm": {
            "time_to_gap_s": el / args.steps,
            "iterations": [r["iterations"] for r in results],
            "pcg_iterations": [r["pcg_iterations"] for r in results],
            "newton_matvecs": [r["newton_matvecs"] for r in results],
            "relgap": results[-1]["relgap"],
            "pobj": results[-1]["pobj"],
        },
        "trajectory": trajectory,
        "newton_apply_loop": {"matvec_per_s": loop_rate, "calls": args.apply_loop},
        "mixed": mixed,
        "roofline": {
            "kernel": ("packed_rows_kernel: A(M), one pass over the packed constraint rows"
                       if kcls == L.SDP_K_A_APPLY else
                       "packed_cols_partial_kernel: A^T(u), one pass over the packed constraint rows"),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_ms": avg_ms,
            "launches": kp["launches"],
            "bytes_per_launch": bytes_per,
        },
        "kernel_time_ms": {"A_apply": prof[L.SDP_K_A_APPLY]["ms"], "AT_apply": prof[L.SDP_K_AT_APPLY]["ms"],
                           "gemm": prof[L.SDP_K_GEMM]["ms"], "newton_apply": prof[L.SDP_K_NEWTON]["ms"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p)
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
