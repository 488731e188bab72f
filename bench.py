"""Benchmark: Newton-operator mat-vecs per second and IPM time to a 1e-8 gap.

Default workload: the matrix-completion SDP n=4000, r=4, m=160000 (entry
sampling), the largest configuration that one GPU holds.  One step = one
FP64 application of the augmented operator of eq. augsys (sdp_newton_apply)
with E Y E on the FP64 matrix cores (Y E as a full n x n x n product, then
the lower triangle of the symmetric E (Y E) mirrored), at a
closed-form centred point (mu = 1e-2, rank-4 split: the shape of the late
iterates; workloads.centred_pair).  value = steps / timed seconds; the
scaling point and its split are prepared before the timed region and every
input is resident in HBM.

The JSON line also carries:
  roofline      the dominant kernel, dgemm_kernel on the full product Y E
                (2 n^3 flops per launch), timed live with HIP events on the
                library's stream;
  forms         the other forms of the same operator (FP64 with the sampled
                A(E Y E), and the FP32 and BF16 forms of the refinement
                sweeps), the preconditioner apply, and the PCG-iteration rate;
  ipm           time to the 1e-8 tolerances from the standard start for the
                fastest FP64 form (sampled) and the BF16-mixed form
                (--solve chooses, FP32-mixed and dense FP64 on request);
  config1       the Gaussian sensing workload n=200, m=2400 (dense A): FP64
                and mixed solves to 1e-8 and its packed-pass HBM roofline;
  cpu_baseline  the CPU oracle's operator at n=4000 on the host cores, and
                the oracle's time to the 1e-8 gap on a reduced completion
                instance of the same generator next to the GPU's.

--workload sensing prints the n=200 line on its own; batched and adjoint
print their own lines.
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
GEMM_KERNEL = "dgemm_kernel<false, false, 128, 128, 0>"
GEMM_COUNTERS_FILE = os.path.join(ROOT, "profiles", "operator_completion_n4000_m160000_counters.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2407_14013_amd", "csrc", "blas.hip")
METRIC = "Newton-op matvecs/s and IPM time-to-1e-8 gap, FP64 vs mixed prec, 1 GPU"
WORKLOAD = "gaussian sensing SDP n=200 r=3 m=2400 (dense A, FP64)"
COMPLETION = "matrix completion SDP n=4000 r=4 m=160000 (entry sampling) at a centred point, mu=1e-2, rank-4 split"
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
REDUCED = (100, 4, 2000)  # reduced completion instance for the oracle's time to gap


def host_threads():
    try:
        from threadpoolctl import threadpool_info

        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count()


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


def gemm_source_digest():
    """SHA-256 of the GEMM sources (the FP64 tiles, their launch plans, the low-precision tiles)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("blas.hip", "launch_plan.hpp", "lowprec.hip"):
        h.update(open(os.path.join(ROOT, "paper_2407_14013_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, record=TRAFFIC_FILE, digest=packed_source_digest):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter runs.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each divided by what the
    same counter read per byte for a device copy of known size in the same run.
    None when no record exists or the kernel source changed since it was taken.
    """
    try:
        rec = json.load(open(record))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != digest() or kernel not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][kernel]
    return 1024.0 * (k["fetch_kib"] / rec["copy"]["fetch_factor"] + k["write_kib"] / rec["copy"]["write_factor"])


def pmc_pass(workload):
    """Short run for the rocprofv3 counter passes: operator products plus a device copy of known size.

    sensing: ten FP64 products on the n=200 sensing workload (packed passes).
    completion: five FP64 and five BF16 products at the centred n=4000
    completion point (the E Y E GEMMs of the default line).
    """
    import torch

    import workloads
    from paper_2407_14013_amd import Context
    from paper_2407_14013_amd import _lib as L

    torch.cuda.set_device(0)
    if workload == "sensing":
        ctx = Context(workloads.config(1))
        N = ctx.aug_dim()
        xin = torch.randn(N, dtype=torch.float64, device="cuda")
        xout = torch.empty_like(xin)
        for _ in range(10):
            ctx.newton_apply(xin, xout)
        ctx.close()
        what = "10 FP64 operator products"
    else:
        p = workloads.config(2)
        X, S, _, _, _ = workloads.centred_pair(p["n"], 4, 1e-2, seed=21)
        Xd, Sd = torch.from_numpy(X).cuda(), torch.from_numpy(S).cuda()
        yd = torch.zeros(p["m"], dtype=torch.float64, device="cuda")
        del X, S
        for prec in (L.SDP_PREC_F64, L.SDP_PREC_BF16):
            with Context(p, inner_prec=prec) as ctx:
                ctx.set_point(Xd, yd, Sd)
                N = ctx.aug_dim()
                xin = torch.randn(N, dtype=torch.float64, device="cuda")
                xout = torch.empty_like(xin)
                for _ in range(5):
                    ctx.newton_apply(xin, xout, prec=None if prec == L.SDP_PREC_F64 else prec)
                torch.cuda.synchronize()
        what = "5 FP64 and 5 BF16 operator products"
    src = torch.randn(64 << 20, dtype=torch.float64, device="cuda")  # 512 MiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"pmc pass ({workload}): {what}, 3 copies of {src.numel() * 8} bytes", flush=True)


def pmc_reduce(out_path, specs):
    """Per-kernel averages (per dispatch) of rocprofv3 counter CSVs: specs are tag=directory pairs."""
    import collections
    import csv
    import glob

    out = {}
    for tag, d in (a.split("=", 1) for a in specs):
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        disp = collections.defaultdict(set)
        for f in glob.glob(f"{d}/**/*counter_collection.csv", recursive=True):
            for row in csv.DictReader(open(f)):
                key = (row["Kernel_Name"][:160], row["Grid_Size"], row["Workgroup_Size"])
                agg[key][row["Counter_Name"]] += float(row["Counter_Value"])
                disp[key].add(row["Dispatch_Id"])
        out[tag] = [{"kernel": k[0], "grid": int(k[1]), "wg": int(k[2]), "dispatches": len(disp[k]),
                     **{c: v / len(disp[k]) for c, v in cs.items()}} for k, cs in agg.items()]
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"reduced {', '.join(f'{k}: {len(v)} kernels' for k, v in out.items())}", flush=True)


def trace_reduce(out_path, trace_dir):
    """Per (kernel, grid) call counts and durations from a rocprofv3 kernel-trace CSV directory."""
    import collections
    import csv
    import glob

    agg = collections.defaultdict(list)
    for f in glob.glob(f"{trace_dir}/**/*kernel_trace.csv", recursive=True):
        for row in csv.DictReader(open(f)):
            dur = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
            # total work-items: Grid_Size, or the product of its per-dimension columns
            grid = 1
            for k, v in row.items():
                if k.startswith("Grid_Size") and v not in ("", None):
                    grid *= int(v)
            agg[(row["Kernel_Name"][:160], grid)].append(dur)
    rows = [{"kernel": k, "grid": g, "calls": len(v), "total_ms": sum(v) / 1e6, "avg_us": sum(v) / len(v) / 1e3,
             "min_us": min(v) / 1e3, "max_us": max(v) / 1e3} for (k, g), v in agg.items()]
    rows.sort(key=lambda r: -r["total_ms"])
    with open(out_path, "w") as fh:
        json.dump(rows, fh, indent=1)
    print(f"reduced {len(rows)} (kernel, grid) pairs", flush=True)


def bench_batched(args):
    """The batched workload: 1024 Gaussian sensing SDPs (n in [16,128], r in {1,2,3}, m = 3nr) in one persistent launch.

    The line's value is the FP32-inner form (the packed rows read in FP32, E Y E
    on the FP32 matrix cores, FP64 refinement of every Newton step); the FP64
    form of the same launch is reported beside it.
    """
    import torch

    import workloads
    from paper_2407_14013_amd import _lib as L
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
    runs = {}
    for name, prec in (("f32_inner", L.SDP_PREC_F32), ("f64", L.SDP_PREC_F64)):
        results, Xs, _ = solve_batched(probs, tune=tune, inner_prec=prec)
        torch.cuda.synchronize()
        launch_ms = results[0]["time_ms"]
        # algorithmic bytes of the packed constraint passes: two passes per operator product,
        # 8 bytes per packed entry in FP64 products, 4 in FP32 ones
        nbytes = 0.0
        for p, r in zip(probs, results):
            N2 = p["n"] * (p["n"] + 1) // 2
            nbytes += 2.0 * p["m"] * N2 * (8.0 * r["newton_matvecs"] + 4.0 * r["lp_matvecs"])
        runs[name] = {
            "launch_ms": launch_ms,
            "instances_per_s": len(probs) / (launch_ms * 1e-3),
            "solved": sum(r["status"] == 0 for r in results),
            "ipm_iterations_total": int(sum(r["iterations"] for r in results)),
            "pcg_iterations_total": int(sum(r["pcg_iterations"] for r in results)),
            "fp64_products": int(sum(r["newton_matvecs"] for r in results)),
            "lowp_products": int(sum(r["lp_matvecs"] for r in results)),
            "a_pass_bytes": nbytes,
            "a_pass_gbs_lower_bound": nbytes / (launch_ms * 1e-3) / 1e9,
        }
        print(f"{name}: {launch_ms / 1e3:.1f} s, {runs[name]['solved']} solved", file=sys.stderr, flush=True)
    head = runs["f32_inner"]
    line = {
        "metric": "IPM time-to-1e-8 gap, batched",
        "value": head["instances_per_s"],
        "unit": "instances/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32 inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": "1024 gaussian sensing SDPs, n in [16,128], r in {1,2,3}, m = 3nr (dense A), "
                               "FP32 inner operator with FP64 refinement"},
        "launch_ms": head["launch_ms"],
        "solved": head["solved"],
        "runs": runs,
        "speedup_f32_inner_vs_f64": runs["f64"]["launch_ms"] / head["launch_ms"],
        "autotune": {"bucket_ms": bucket_ms, "configs": sorted({(t.rows_per_wave, t.aq_group, t.gemm_tile) for t in tune})},
        "generate_s": gen_s,
    }
    if not args.no_cpu_baseline:
        from oracle import ipm

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
            "cores": host_threads(),
            "kind": "oracle",
            "sample": f"{len(sample)} instances spread over the size range solved by the oracle in {el:.1f} s, "
                      f"scaled to the whole batch by sum(m n^2)",
        }
    print(json.dumps(line))


# Table rmc and Table snl rows (n, m, m_o) with the paper's own times for its
# method (CPU, another machine): context, not a target on this hardware
RMC_ROWS = [(100, 3000, 12, 1.2), (300, 45000, 150, 32.1), (500, 125000, 300, 127.0), (1000, 500000, 450, 1106.0)]
SNL_ROWS = [(50, 1000, 30, 1.0), (50, 1300, 50, 0.6), (100, 5000, 100, 4.1), (300, 45000, 300, 117.5),
            (500, 100000, 420, 499.3), (550, 110000, 460, 559.4), (500, 120000, 500, 760.5)]


def bench_lp(args, which):
    """Time to the 1e-8 tolerances on the experiments' RMC or SNL instances (LP cone block).

    RMC: entry-sampling rows plus slack pairs (eq. rmc-sdp), m sampled svec
    entries of X* = G G^T (G n x 2, N(0, 10^2)), m_o outliers N(0, 10^4).
    SNL: n sensors, 3 anchors in [0, 1]^2, distance rows (sparse constraint
    kind) plus slack pairs (eq. snl-sdp), min(3n, m/8) anchor-sensor measurements and the rest
    between sensors, m_o outliers N(0, I) inside the norm, split in proportion.  One solve per row from the
    standard start, timed around sdp_solve; the recovery error is
    ||X - X*||_F / ||X*||_F (RMC) or ||Y - Y*||_F (SNL) on the host.
    """
    import torch

    import workloads
    from paper_2407_14013_amd import Context

    torch.cuda.set_device(0)
    rows = []
    for row in (RMC_ROWS if which == "rmc" else SNL_ROWS):
        n, m, m_o, paper_s = row
        t0 = time.perf_counter()
        if which == "rmc":
            p = workloads.robust_completion(n, m, m_o, seed=100 + n)
        else:
            m_a = min(3 * n, m // 8)  # anchor-sensor pairs (there are only 3 n of them)
            m_ao = m_o * m_a // m
            p = workloads.sensor_localization(n, m - m_a, m_a, m_o - m_ao, m_ao, seed=100 + n + m, kind="sparse")
        gen_s = time.perf_counter() - t0
        with Context(p) as ctx:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve(raise_on_stall=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            X = ctx.get_point()[0].cpu().numpy()
        if which == "rmc":
            rec = float(np.linalg.norm(X - p["Xstar"]) / np.linalg.norm(p["Xstar"]))
        else:
            rec = float(np.linalg.norm(X[: p["d"], p["d"]:] - p["Ystar"]))
        rec_row = {"n": n, "m": m, "m_o": m_o, "time_to_gap_s": el, "status": res["status"],
                   "iterations": res["iterations"], "pcg_iterations": res["pcg_iterations"],
                   "relgap": res["relgap"], "pinf": res["pinf"], "dinf": res["dinf"], "recovery_error": rec,
                   "paper_cpu_s": paper_s, "generate_s": gen_s}
        rows.append(rec_row)
        print(f"{which} n={n} m={m} m_o={m_o}: {el:.2f} s, {res['iterations']} its, status {res['status']}, "
              f"recovery {rec:.1e}", file=sys.stderr, flush=True)
    total = sum(r["time_to_gap_s"] for r in rows)
    line = {
        "metric": f"IPM time-to-1e-8 gap, {which.upper()} table instances",
        "value": len(rows) / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("robust matrix completion (eq. rmc-sdp), rank 2, entry sampling + LP slack pairs"
                                if which == "rmc" else
                                "sensor network localization with outliers (eq. snl-sdp), d = 2, 3 anchors, "
                                "sparse distance rows + LP slack pairs")},
        "rows": rows,
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


def sensing_line(args, steps, warmup, with_cpu=True, with_mixed=True):
    """The n=200 dense Gaussian sensing workload: FP64 solves to 1e-8, mixed solves, packed-pass roofline."""
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

    for _ in range(warmup):
        one_solve()
    torch.cuda.synchronize()
    ctx.profile_enable([L.SDP_K_A_APPLY, L.SDP_K_AT_APPLY])
    results = []
    t0 = time.perf_counter()
    for _ in range(steps):
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
    if with_mixed:
        for name, prec in (("f32", L.SDP_PREC_F32), ("bf16", L.SDP_PREC_BF16)):
            mctx = Context(p, inner_prec=prec)

            def msolve():
                mctx.set_point(X0, y0, S0)
                return mctx.solve()

            for _ in range(warmup):
                msolve()
            torch.cuda.synchronize()
            mres = []
            tm0 = time.perf_counter()
            for _ in range(steps):
                mres.append(msolve())
            torch.cuda.synchronize()
            mel = time.perf_counter() - tm0
            mctx.close()
            for r in mres:
                assert r["status"] == 0 and r["relgap"] <= 1e-8, r
            mixed[name] = {
                "time_to_gap_s": mel / steps,
                "speedup_vs_fp64": el / mel,
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
        "value": matvecs / el,
        "unit": "matvec/s",
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": el * 1e3 / steps,
        "dtype": "f64",
        "config": {"workload": WORKLOAD, "precision": "fp64", "ipm_tol": 1e-8, "inner_tol": 1e-10},
        "ipm": {
            "time_to_gap_s": el / steps,
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
            "traffic": measured_traffic(kname),
            "avg_launch_ms": avg_ms,
            "launches": kp["launches"],
            "bytes_per_launch": bytes_per,
        },
        "kernel_time_ms": {"A_apply": prof[L.SDP_K_A_APPLY]["ms"], "AT_apply": prof[L.SDP_K_AT_APPLY]["ms"],
                           "gemm": prof[L.SDP_K_GEMM]["ms"], "newton_apply": prof[L.SDP_K_NEWTON]["ms"]},
    }
    if with_cpu:
        line["cpu_baseline"] = cpu_baseline(p)
    ctx.close()
    return line


# name: context options (inner precision, sampled A(E Y E) for the FP64 products, refinement mode)
SOLVE_FORMS = {
    "f64_sampled": {"inner_prec": 0, "sparse_sandwich": 1},
    "f64": {"inner_prec": 0},
    "f32": {"inner_prec": 1},
    "bf16": {"inner_prec": 2},
    "bf16_replace": {"inner_prec": 2, "refine_mode": 1},
    "bf16_replace_sampled": {"inner_prec": 2, "refine_mode": 1, "sparse_sandwich": 1},
    "f32_replace_sampled": {"inner_prec": 1, "refine_mode": 1, "sparse_sandwich": 1},
}


def completion_line(args):
    """The n=4000 matrix-completion workload: operator rate, its roofline, and the solves to 1e-8."""
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
    flops = 2.0 * n ** 3  # the n x n x n product Y E
    print("completion workload generated", file=sys.stderr, flush=True)

    def xin_for(N):
        return torch.randn(N, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(0))

    def time_precond(ctx, xin, xout, reps=20):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.precond_apply(xin, xout)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    # ---- the headline: FP64 operator with the dense E Y E products ----------------------
    with Context(p) as ctx:
        ctx.set_point(Xd, yd, Sd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sc = ctx.get_scaling()  # prepares the scaling point and its split (not timed below)
        torch.cuda.synchronize()
        t_scaling = time.perf_counter() - t0
        N = ctx.aug_dim()
        xin = xin_for(N)
        xout = torch.empty_like(xin)
        for _ in range(args.warmup):
            ctx.newton_apply(xin, xout)
        torch.cuda.synchronize()
        ctx.profile_enable([L.SDP_K_SANDWICH, L.SDP_K_SANDWICH_LOWER])
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.newton_apply(xin, xout)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sw = ctx.profile_get(L.SDP_K_SANDWICH)
        swl = ctx.profile_get(L.SDP_K_SANDWICH_LOWER)
        ctx.profile_enable([])
        prec_ms = time_precond(ctx, xin, xout)
    avg_ms = sw["ms"] / max(sw["launches"], 1)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    op_ms = 1e3 * el / args.steps
    forms = {"f64": {"ms_per_matvec": op_ms, "matvec_per_s": args.steps / el, "precond_apply_ms": prec_ms,
                     "pcg_iterations_per_s": 1e3 / (op_ms + prec_ms), "scaling_setup_s": t_scaling,
                     "r": sc["r"], "d": N - m,
                     "sandwich_gemm": {"launches": sw["launches"], "avg_launch_ms": avg_ms,
                                       "achieved_tflops": achieved, "peak_tflops": MFMA_PEAK_TFLOPS["f64"],
                                       "frac": achieved / MFMA_PEAK_TFLOPS["f64"]}}}
    if swl["launches"]:
        # E (Y E): n (n + 1) / 2 entries of 2 n flops each (the strip's extra entries not counted)
        lms = swl["ms"] / swl["launches"]
        ltf = n * n * (n + 1.0) / (lms * 1e-3) / 1e12
        forms["f64"]["sandwich_lower"] = {"launches": swl["launches"], "avg_launch_ms": lms,
                                          "algorithmic_flops": n * n * (n + 1.0), "achieved_tflops": ltf,
                                          "frac": ltf / MFMA_PEAK_TFLOPS["f64"]}
    lower_note = (f", E (Y E) lower triangle {forms['f64']['sandwich_lower']['avg_launch_ms']:.3f} ms"
                  if "sandwich_lower" in forms["f64"] else "")
    print(f"f64: {op_ms:.3f} ms per operator product, Y E GEMM {achieved:.1f} TFLOP/s{lower_note}, "
          f"preconditioner {prec_ms:.3f} ms", file=sys.stderr, flush=True)

    # ---- the other forms of the same operator ---------------------------------------------
    for name in [f for f in args.forms.split(",") if f and f != "f64"]:
        fo = SOLVE_FORMS[name]
        prec, sparse = fo["inner_prec"], fo.get("sparse_sandwich", 0)
        with Context(p, inner_prec=prec, sparse_sandwich=sparse) as ctx:
            ctx.set_point(Xd, yd, Sd)
            ctx.get_scaling()
            N = ctx.aug_dim()
            xin = xin_for(N)
            xout = torch.empty_like(xin)
            pr = None if prec == 0 else prec
            for _ in range(3):
                ctx.newton_apply(xin, xout, prec=pr)
            torch.cuda.synchronize()
            classes = [L.SDP_K_SAMPLED_YE, L.SDP_K_SAMPLED_DOTS] if sparse else [L.SDP_K_SANDWICH]
            ctx.profile_enable(classes)
            calls = args.form_loop
            t0 = time.perf_counter()
            for _ in range(calls):
                ctx.newton_apply(xin, xout, prec=pr)
            torch.cuda.synchronize()
            fel = time.perf_counter() - t0
            prof = {k: ctx.profile_get(k) for k in classes}
            ctx.profile_enable([])
            pms = time_precond(ctx, xin, xout)
        fms = 1e3 * fel / calls
        f = {"ms_per_matvec": fms, "matvec_per_s": calls / fel, "precond_apply_ms": pms,
             "pcg_iterations_per_s": 1e3 / (fms + pms)}
        if sparse:
            # both sampled kernels at algorithmic HBM bytes (each operand read once)
            for key, k in (("sampled_ye", L.SDP_K_SAMPLED_YE), ("sampled_dots", L.SDP_K_SAMPLED_DOTS)):
                pk = prof[k]
                gbs = pk["bytes"] / (pk["ms"] * 1e-3) / 1e9
                f[key] = {"launches": pk["launches"], "avg_launch_ms": pk["ms"] / pk["launches"],
                          "bytes_per_launch": pk["bytes"] / pk["launches"], "achieved_gbs": gbs,
                          "peak_gbs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS}
            note = f"Y E {f['sampled_ye']['avg_launch_ms']:.3f} ms, dots {f['sampled_dots']['avg_launch_ms']:.3f} ms"
        else:
            pk = prof[L.SDP_K_SANDWICH]
            tf = flops * pk["launches"] / (pk["ms"] * 1e-3) / 1e12
            f["sandwich_gemm"] = {"launches": pk["launches"], "avg_launch_ms": pk["ms"] / pk["launches"],
                                  "achieved_tflops": tf, "peak_tflops": MFMA_PEAK_TFLOPS[name],
                                  "frac": tf / MFMA_PEAK_TFLOPS[name]}
            note = f"E Y E GEMM {tf:.1f} TFLOP/s"
        forms[name] = f
        print(f"{name}: {fms:.3f} ms per operator product, {note}, preconditioner {pms:.3f} ms", file=sys.stderr,
              flush=True)
    del Xd, Sd, yd

    line = {
        "metric": METRIC,
        "value": args.steps / el,
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": op_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": COMPLETION, "step": "one FP64 augmented-operator product, E Y E on the FP64 "
                                                   "MFMA: Y E, then the lower triangle of E (Y E)"},
        "roofline": {
            "kernel": GEMM_KERNEL + ": the n x n x n product Y E of E Y E",
            "bound": "mfma",
            "achieved": achieved,
            "peak": MFMA_PEAK_TFLOPS["f64"],
            "unit": "TFLOP/s",
            "frac": achieved / MFMA_PEAK_TFLOPS["f64"],
            "traffic": measured_traffic(GEMM_KERNEL, GEMM_COUNTERS_FILE, gemm_source_digest),
            "flops_per_launch": flops,
            "avg_launch_ms": avg_ms,
            "launches": sw["launches"],
        },
        "forms": forms,
    }

    # ---- solves to the 1e-8 tolerances from the standard start ---------------------------
    solves = {}
    for name in [f for f in args.solve.split(",") if f]:
        with Context(p, verbose=1 if args.verbose else 0, **SOLVE_FORMS[name]) as ctx:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve(raise_on_stall=False)
            torch.cuda.synchronize()
            solves[name] = {"time_to_gap_s": time.perf_counter() - t0, "status": res["status"],
                            "iterations": res["iterations"], "pcg_iterations": res["pcg_iterations"],
                            "fp64_matvecs": res["newton_matvecs"], "lowp_matvecs": res["lp_matvecs"],
                            "relgap": res["relgap"], "pinf": res["pinf"], "dinf": res["dinf"], "pobj": res["pobj"]}
        print(f"solve {name}: {solves[name]}", file=sys.stderr, flush=True)
    if solves:
        fp64 = [k for k in solves if k.startswith("f64")]
        best = min(fp64, key=lambda k: solves[k]["time_to_gap_s"]) if fp64 else None
        for k, v in solves.items():
            if best and not k.startswith("f64"):
                v["speedup_vs_best_fp64"] = solves[best]["time_to_gap_s"] / v["time_to_gap_s"]
                v["pobj_rel_diff_vs_fp64"] = abs(v["pobj"] - solves[best]["pobj"]) / abs(solves[best]["pobj"])
        line["ipm"] = {"best_fp64_form": best, **solves}

    if not args.no_config1:
        c1 = sensing_line(args, steps=3, warmup=1, with_cpu=False)
        line["config1"] = c1
        print(f"config 1: {c1['ms_per_step']:.1f} ms to the 1e-8 gap", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = completion_cpu_baseline(p, x, s, V, r0)
    return line


def completion_cpu_baseline(p, x, s, V, r0, budget_s=15.0):
    """The oracle's operator at n=4000 (same point) and its time to gap on a reduced instance, beside the GPU's."""
    import torch

    import workloads
    from oracle import ipm, reform as rf
    from paper_2407_14013_amd import Context

    n, m = p["n"], p["m"]
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
    while time.perf_counter() - t0 < budget_s:
        rf.aug_apply(p, sp, E, sig, xh[:m], xh[m:])
        calls += 1
    el = time.perf_counter() - t0
    # time to gap: the oracle's direct method on a reduced instance of the same generator
    nr, rr, mr = REDUCED
    q = workloads.matrix_completion(nr, rr, mr, seed=2)
    t0 = time.perf_counter()
    ores = ipm.solve(q)
    o_s = time.perf_counter() - t0
    with Context(q) as ctx:
        start = [t.clone() for t in ctx.get_point()]
        ctx.solve()  # warm-up (first use of the kernels at this size)
        ctx.set_point(*start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gres = ctx.solve()
        torch.cuda.synchronize()
        g_s = time.perf_counter() - t0
    return {
        "value": calls / el,
        "unit": "matvec/s",
        "cores": host_threads(),
        "kind": "oracle",
        "sample": f"{calls} applications of the oracle's augmented operator (Section 5 products) on the same "
                  f"workload and point, split supplied in closed form, {el:.1f} s",
        "time_to_gap": {"instance": f"matrix completion n={nr} r={rr} m={mr} (same generator)",
                        "oracle_s": o_s, "oracle_iterations": ores["iterations"],
                        "oracle_pobj": ores["history"][-1]["pobj"], "gpu_fp64_s": g_s,
                        "gpu_iterations": gres["iterations"], "gpu_pobj": gres["pobj"]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--apply-loop", type=int, default=200, help="sensing: operator products in the tight loop")
    ap.add_argument("--form-loop", type=int, default=50, help="completion: products timed per extra form")
    ap.add_argument("--pmc-pass", choices=["sensing", "completion"], default=None,
                    help="only the short run profiled for hardware counters")
    ap.add_argument("--pmc-reduce", nargs="+", metavar="ARG", default=None,
                    help="OUT.json tag=dir ...: per-kernel averages of rocprofv3 counter CSVs (no GPU)")
    ap.add_argument("--trace-reduce", nargs=2, metavar=("OUT", "DIR"), default=None,
                    help="per (kernel, grid) durations from a rocprofv3 kernel-trace CSV directory (no GPU)")
    ap.add_argument("--no-mixed", action="store_true", help="sensing: skip the mixed-precision solves")
    ap.add_argument("--no-config1", action="store_true", help="completion: skip the n=200 sensing solves")
    ap.add_argument("--workload", choices=["completion", "sensing", "batched", "adjoint", "rmc", "snl"],
                    default="completion",
                    help="completion: the headline line (n=4000 entry sampling); sensing: the n=200 dense line; "
                         "batched: 1024 small SDPs in one launch; adjoint: n=1000 completion forward + backward; "
                         "rmc / snl: the experiments' table instances with the LP cone block")
    ap.add_argument("--verbose", action="store_true", help="completion: one line per interior-point iteration")
    ap.add_argument("--forms", default="f64,f64_sampled,f32,bf16",
                    help="completion: operator forms to time (comma list of f64, f64_sampled, f32, bf16)")
    ap.add_argument("--solve", default="f64_sampled,bf16",
                    help="completion: solves to time to the 1e-8 tolerances (comma list of "
                         + ", ".join(SOLVE_FORMS) + "; empty for none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every instance of this workload fits one MI355X, "
              "and the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.pmc_reduce:
        pmc_reduce(args.pmc_reduce[0], args.pmc_reduce[1:])
        return
    if args.trace_reduce:
        trace_reduce(*args.trace_reduce)
        return
    if args.pmc_pass:
        pmc_pass(args.pmc_pass)
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "adjoint":
        bench_adjoint(args)
        return
    if args.workload in ("rmc", "snl"):
        bench_lp(args, args.workload)
        return
    if args.workload == "completion":
        print(json.dumps(completion_line(args)))
        return
    line = sensing_line(args, args.steps, args.warmup, with_cpu=not args.no_cpu_baseline,
                        with_mixed=not args.no_mixed)
    line = {"metric": METRIC, "value": line.pop("value"), "unit": line.pop("unit"), "n_gpus": 1,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic", **line}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
