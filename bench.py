"""Benchmark: H^2 construction of the 131072-point exponential-covariance cube.

One step = one complete h2_build (Algorithm 1 with adaptive sampling: tree and
lists, Gaussian draw, dense on-the-fly sketch, near-field generation and
subtraction, convergence tests, IDs, upsweeps, coupling generation) with the
points already resident in HBM.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H2 build time (N=131072, tol 1e-6) + sketch TFLOP/s; mixed vs FP64 speedup"
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector (= FP64 matrix) peak


def sketch_flops_per_entry(dim: int, ncols: int) -> float:
    """Algorithmic FP64 operations per kernel entry of the fused sketch:
    generation = dim differences + (2 dim - 1) square-accumulate + sqrt + scale + exp,
    contraction = 2 * ncols (one multiply-add per output column)."""
    return (3 * dim - 1 + 3) + 2 * ncols


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (profiles/sketch_traffic.json), or None when the kernel sources changed
    since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "sketch_traffic.json")))
        csrc = os.path.join(ROOT, "paper_2506_16759_amd", "csrc")
        src = hashlib.sha256(open(os.path.join(csrc, "h2_kernels.hip"), "rb").read()
                             + open(os.path.join(csrc, "h2_devmath.hpp"), "rb").read()).hexdigest()
        if rec.get("source_sha256") != src or kernel not in rec["kernels"]:
            return None
        k = rec["kernels"][kernel]
        return k["fetch_bytes"] + k["write_bytes"]
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(w, samples_used: int, rows: int = 2048):
    """The oracle's dense sketch on a sample of rows, scaled to the full pass count."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.kernels import KernelOperator
    from oracle.philox import gaussian

    pts = w.points()
    op = KernelOperator(pts, w.kernel, w.length)
    sel = np.arange(rows)
    omega = gaussian(w.omega_seed, np.arange(w.n), 0, w.d0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        op.sketch_rows(sel, omega)
        dt = time.perf_counter() - t0
    per_pass_full = dt * (w.n / rows)
    # the build draws d0 columns, then d_inc per adaptive round; every pass costs the same
    passes = 1 + max(0, samples_used - w.d0) // w.d_inc
    return {
        "value": per_pass_full * passes,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle dense sketch of {rows} of {w.n} rows x {w.d0} columns ({dt:.2f} s), scaled to all rows "
                   f"and the build's {passes} sketch passes; the oracle's O(N) steps are not included, so this is "
                   f"a lower bound on its build time"),
    }


def bench_batched(h2, ctx, steps: int = 2):
    """The 64-problem covariance batch: batched FP64 and FP32 builds (one
    hipGraph each) against 64 sequential single FP64 builds."""
    import torch

    from paper_2506_16759_amd.workloads import batch_problems
    ws = batch_problems()
    probs = [dict(points=torch.from_numpy(w.points()).cuda(), kernel=w.kernel, length=w.length,
                  leaf_size=w.leaf_size, tol=w.tol, eta=w.eta, d0=w.d0, d_inc=w.d_inc, seed=w.omega_seed)
             for w in ws]
    res = {"problems": len(ws), "total_n": int(sum(w.n for w in ws)),
           "sum_n2": float(sum(float(w.n) ** 2 for w in ws))}
    t0 = time.perf_counter()
    leaves = h2.autotune_leaf(ctx, probs, candidates=(32, 64, 128), d_max=96)
    res["autotune_ms"] = (time.perf_counter() - t0) * 1e3
    res["leaf_sizes"] = {str(c): leaves.count(c) for c in (32, 64, 128)}
    for p, leaf in zip(probs, leaves):
        p["leaf_size"] = leaf
    for name, prec in (("fp64", h2.FP64), ("bf16x6", h2.BF16X6)):
        times, info = [], None
        for i in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                mats, info = h2.build_batched(ctx, probs, precision=prec, d_max=96, return_info=True)
            except h2.H2Error as exc:
                res[name] = {"error": str(exc)}
                break
            torch.cuda.synchronize()
            if i > 0:
                times.append((time.perf_counter() - t0) * 1e3)
            samples = [m.info()["samples"] for m in mats]
            for m in mats:
                m.close()
            print(f"[bench] batched {name} {times[-1] if times else 0:.1f} ms", file=sys.stderr, flush=True)
        else:
            res[name] = {"ms_per_batch": statistics.median(times), "device_ms": info["t_device_ms"],
                         "plan_ms": info["t_plan_ms"], "setup_ms": info["t_setup_ms"],
                         "alloc_ms": info["t_alloc_ms"], "results_ms": info["t_results_ms"],
                         "capture_ms": info["t_capture_ms"], "graph_nodes": info["graph_nodes"],
                         "device_gb": info["device_bytes"] / 1e9,
                         "first_pass_columns": info["first_pass"], "second_pass_problems": info["second_pass"],
                         "samples_range": [min(samples), max(samples)]}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in probs:
        H = h2.build(ctx, p["points"], p["kernel"], p["length"], tol=p["tol"], leaf_size=p["leaf_size"],
                     eta=p["eta"], d0=p["d0"], d_inc=p["d_inc"], seed=p["seed"])
        H.close()
    torch.cuda.synchronize()
    res["sequential_fp64_ms"] = (time.perf_counter() - t0) * 1e3
    if "ms_per_batch" in res.get("fp64", {}):
        res["batched_vs_sequential_speedup"] = res["sequential_fp64_ms"] / res["fp64"]["ms_per_batch"]
        if "ms_per_batch" in res.get("bf16x6", {}):
            res["mixed_vs_fp64_batched_speedup"] = res["fp64"]["ms_per_batch"] / res["bf16x6"]["ms_per_batch"]
    return res


def bench_update(h2, ctx, n: int = 1 << 17):
    """Low-rank update of an H^2 matrix (rank 64) on n points: build H, then
    the two-sided update with H's matvec as the black box.  The error is
    measured against that black box, (H + U V^T) x, on two Gaussian vectors."""
    import torch

    from paper_2506_16759_amd.workloads import cube_update
    w = cube_update(n)
    b = w.base
    pts = torch.from_numpy(b.points()).cuda()
    H = h2.build(ctx, pts, b.kernel, b.length, tol=b.tol, leaf_size=b.leaf_size, eta=b.eta, d0=b.d0,
                 d_inc=b.d_inc, seed=b.omega_seed)
    U, V = w.factors()
    Ut, Vt = torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda()
    times = []
    for i in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Hu = h2.build_update(ctx, H, Ut, Vt, tol=w.tol, d0=w.d0, d_inc=w.d_inc, d_max=w.d_max, seed=w.omega_seed,
                             oversample=w.oversample)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        info = Hu.info()
        if i == 0:
            Hu.close()
    x = torch.randn(2, n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5)).T
    ref = H.matvec(x) + Ut @ (Vt.T @ x)
    err = float(torch.linalg.norm(Hu.matvec(x) - ref) / torch.linalg.norm(ref))
    print(f"[bench] update n={n} {times[-1]:.1f} ms error {err:.2e}", file=sys.stderr, flush=True)
    out = {"workload": w.name, "n": n, "rank": w.rank, "ms_per_update": times[-1], "error_vs_sampler": err,
           "old_build_ms": H.info()["t_total"], "samples": info["samples"], "rounds": info["rounds"],
           "rank_range": [info["rank_min"], info["rank_max"]],
           "phases_ms": {k[2:]: round(info[k], 3) for k in info if k.startswith("t_")}}
    Hu.close()
    H.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sketch-launches", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 64-problem batched build and the low-rank update measurements")
    ap.add_argument("--only-extras", action="store_true",
                    help="only the 64-problem batched build and the low-rank update (printed as one JSON line)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only run the sketch (FP64, FP32, bf16x3, FP32E, bf16x6; 32 columns) twice each and a 1 GiB copy of "
                         "known size, for counter collection")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2506_16759_amd as h2
    from paper_2506_16759_amd.workloads import CUBE_131K

    w = CUBE_131K
    tol = args.tol if args.tol is not None else w.tol
    if args.profile_kernels:
        ctx = h2.Context(0)
        pts = torch.from_numpy(w.points()).cuda()
        omega = h2.gaussian(ctx, w.omega_seed, torch.arange(w.n, dtype=torch.int32), 0, w.d0)
        for prec in (h2.FP64, h2.FP32, h2.BF16X3, h2.FP32E, h2.BF16X6):
            for _ in range(2):
                h2.sketch(ctx, pts, w.kernel, w.length, omega, precision=prec)
        # calibration: a plain device copy of exactly 1 GiB (reads 1 GiB, writes 1 GiB)
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_kernels": "done", "copy_bytes": a.numel() * 8}), flush=True)
        return
    if args.only_extras:
        ctx = h2.Context(0)
        upd = bench_update(h2, ctx)
        print(json.dumps({"update": upd, "batched": bench_batched(h2, ctx)}), flush=True)
        return
    print(f"[bench] workload {w.name} n={w.n} tol={tol}", file=sys.stderr, flush=True)
    ctx = h2.Context(0)
    pts = torch.from_numpy(w.points()).cuda()
    opts = h2.opts_default(tol=tol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0, d_inc=w.d_inc, seed=w.omega_seed)

    def timed_builds(o, label, steps, warmup):
        infos = []
        for i in range(warmup):
            H = h2.build(ctx, pts, w.kernel, w.length, opts=o)
            infos.append(H.info())
            H.close()
            print(f"[bench] {label} warmup {i} {infos[-1]['t_total']:.1f} ms", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        times = []
        t0 = time.perf_counter()
        for i in range(steps):
            ts = time.perf_counter()
            H = h2.build(ctx, pts, w.kernel, w.length, opts=o)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
            infos.append(H.info())
            H.close()
            print(f"[bench] {label} step {i} {times[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3, times, infos[-1]

    ms_per_step, times, info = timed_builds(opts, "fp64", args.steps, args.warmup)

    # mixed precision on the same points at the same tolerance: three-term
    # split bf16 products (bf16x6), FP32 matrix cores (fp32), FP32 entries
    # contracted in FP64 (fp32e); bf16x3 at tol 1e-4 (its products carry
    # ~2^-17 relative error), with FP64 at 1e-4 for comparison
    mixed = {}
    for name, prec, mtol in (("bf16x6", h2.BF16X6, tol), ("fp32", h2.FP32, tol), ("fp32e", h2.FP32E, tol),
                             ("fp64_tol1e-4", h2.FP64, 1e-4), ("bf16x3_tol1e-4", h2.BF16X3, 1e-4)):
        o = h2.opts_default(tol=mtol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0, d_inc=w.d_inc, seed=w.omega_seed,
                            precision=prec)
        try:
            mms, mtimes, minfo = timed_builds(o, name, max(1, args.steps // 2 + 1), 1)
            mixed[name] = {"tol": mtol, "ms_per_build": mms, "samples": minfo["samples"],
                           "adaptive_rounds": minfo["rounds"], "rank_range": [minfo["rank_min"], minfo["rank_max"]],
                           "sketch_phase_ms": minfo["t_sample"]}
            if mtol == tol:
                mixed[name]["speedup_vs_fp64"] = ms_per_step / mms
        except h2.H2Error as exc:
            mixed[name] = {"tol": mtol, "error": str(exc)}
    if "ms_per_build" in mixed.get("bf16x3_tol1e-4", {}) and "ms_per_build" in mixed.get("fp64_tol1e-4", {}):
        mixed["bf16x3_tol1e-4"]["speedup_vs_fp64"] = (mixed["fp64_tol1e-4"]["ms_per_build"]
                                                      / mixed["bf16x3_tol1e-4"]["ms_per_build"])

    # dominant kernel: the fused sketch, timed live on the library's stream
    nc = w.d0
    omega = h2.gaussian(ctx, w.omega_seed, torch.arange(w.n, dtype=torch.int32), 0, nc)
    h2.sketch(ctx, pts, w.kernel, w.length, omega)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(ctx.stream)
    for _ in range(args.sketch_launches):
        h2.sketch(ctx, pts, w.kernel, w.length, omega)
    ev1.record(ctx.stream)
    ev1.synchronize()
    sk_ms = ev0.elapsed_time(ev1) / args.sketch_launches
    # the same sketch with three-term split bf16 products
    h2.sketch(ctx, pts, w.kernel, w.length, omega, precision=h2.BF16X6)
    ev0.record(ctx.stream)
    for _ in range(args.sketch_launches):
        h2.sketch(ctx, pts, w.kernel, w.length, omega, precision=h2.BF16X6)
    ev1.record(ctx.stream)
    ev1.synchronize()
    sk6_ms = ev0.elapsed_time(ev1) / args.sketch_launches
    entries = float(w.n) * w.n
    achieved = sketch_flops_per_entry(w.dim, nc) * entries / (sk_ms * 1e-3) / 1e12
    sketch_tflops = 2.0 * entries * nc / (sk_ms * 1e-3) / 1e12

    out = {
        "metric": METRIC,
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "dim": w.dim, "kernel": f"exp(-r/{w.length})",
                   "leaf_size": w.leaf_size, "eta": w.eta, "tol": tol, "d0": w.d0, "d_inc": w.d_inc,
                   "precision": "fp64"},
        "median_step_ms": statistics.median(times) * 1e3,
        "sketch_tflops": sketch_tflops,
        "sketch_entries_per_s": entries / (sk_ms * 1e-3),
        "sketch_kernel_ms": sk_ms,
        "sketch_bf16x6_kernel_ms": sk6_ms,
        "sketch_bf16x6_tflops": 2.0 * entries * nc / (sk6_ms * 1e-3) / 1e12,
        "mixed_vs_fp64_speedup": mixed.get("bf16x6", {}).get("speedup_vs_fp64"),
        "mixed": mixed,
        "samples": info["samples"],
        "adaptive_rounds": info["rounds"],
        "rank_range": [info["rank_min"], info["rank_max"]],
        "phases_ms": {k[2:]: round(info[k], 3) for k in info if k.startswith("t_")},
        "bytes": {"dense": info["bytes_dense"], "coupling": info["bytes_coupling"], "basis": info["bytes_basis"]},
        "roofline": {
            "kernel": "sketch_f64_kernel<3,exp,32>",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic("sketch_f64_kernel<3,exp,32>"),
        },
    }
    if not args.no_extras:
        # the update first: its 27 GB of couplings would otherwise wait for the
        # memory pool to map new pages past what the batched builds left cached
        out["update"] = bench_update(h2, ctx)
        out["batched"] = bench_batched(h2, ctx)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, info["samples"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
