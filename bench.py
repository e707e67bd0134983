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


def sketch_source_digest() -> str:
    """SHA-256 of the sources the sketch kernels are compiled from: h2_kernels.hip
    up to the block generator (helpers, Philox, the FP64 and reduced-precision
    sketch kernels), its sketch launcher, and h2_devmath.hpp."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2506_16759_amd", "csrc")
    text = open(os.path.join(csrc, "h2_kernels.hip")).read()
    head = text[:text.index("// ------------------------------------------------------ kernel block gen")]
    i = text.index("hipError_t sketch(hipStream_t s, int precision")
    j = text.index("\nhipError_t ", i + 1)
    math = open(os.path.join(csrc, "h2_devmath.hpp")).read()
    return hashlib.sha256((head + text[i:j] + math).encode()).hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (profiles/sketch_traffic.json), or None when the sketch sources changed
    since the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "sketch_traffic.json")))
        if rec.get("source_sha256") != sketch_source_digest() or kernel not in rec["kernels"]:
            return None
        k = rec["kernels"][kernel]
        return k["fetch_bytes"] + k["write_bytes"]
    except (OSError, ValueError, KeyError):
        return None


def traffic_summary(fetch_dir: str, write_dir: str, sq_dir: str | None = None) -> dict:
    """HBM bytes per sketch launch from two rocprofv3 --pmc runs of
    --profile-kernels (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
    scaled by what the same counter reads for the run's 1 GiB copy; the first
    launch of each 64-column sketch kernel counts.  With a third run's
    directory (SQ counters of the same command), its counters of the same
    dispatches are attached as "sq"."""
    import csv
    import glob
    import re

    def load(d, counter):
        rows = list(csv.DictReader(open(glob.glob(os.path.join(d, "*counter_collection.csv"))[0])))
        out = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            k = int(r["Dispatch_Id"])
            name, val = out.get(k, (r["Kernel_Name"], 0.0))
            out[k] = (name, val + float(r["Counter_Value"]))
        return out

    def short(name):
        m = re.search(r"::(\w+)(<[^>]*>)?\(", name)
        return (m.group(1) + (m.group(2) or "").replace(" ", "")) if m else name[:40]

    f, w = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    # the 1 GiB copy is the largest copy of the run
    fs = gib_kib / max(v for n, v in f.values() if "copyBuffer" in n)
    ws = gib_kib / max(v for n, v in w.values() if "copyBuffer" in n)
    names = {"sketch_f64_kernel<3,1,64>": "sketch_f64_kernel<3,exp,64>",
             "sketch_f32_kernel<3,1,64>": "sketch_f32_kernel<3,exp,64>",
             "sketch_bf16_kernel<3,1,64,2>": "sketch_bf16_kernel<3,exp,64,2>",
             "sketch_e32_kernel<3,1,64>": "sketch_e32_kernel<3,exp,64>",
             "sketch_bf16_kernel<3,1,64,3>": "sketch_bf16_kernel<3,exp,64,3>",
             "sketch_sym_f64_kernel<3,1>": "sketch_sym_f64_kernel<3,exp>",
             "sketch_sym_reduce_kernel": "sketch_sym_reduce_kernel"}
    q = _load_pmc(sq_dir) if sq_dir else {}
    kernels = {}
    for k in sorted(f):
        n = names.get(short(f[k][0]))
        if n and n not in kernels and k in w:
            kernels[n] = {"fetch_bytes": f[k][1] * fs * 1024, "write_bytes": w[k][1] * ws * 1024}
            if k in q:
                kernels[n]["sq"] = q[k]["c"]
    return {"source_sha256": sketch_source_digest(), "fetch_scale": fs, "write_scale": ws, "kernels": kernels}


def _load_pmc(d: str):
    """Per dispatch of one rocprofv3 --pmc run: kernel name, counters (summed
    over dimensions) and the kernel-trace duration in ms."""
    import csv
    import glob
    out = {}
    for r in csv.DictReader(open(glob.glob(os.path.join(d, "*counter_collection.csv"))[0])):
        k = int(r["Dispatch_Id"])
        e = out.setdefault(k, {"name": r["Kernel_Name"], "c": {}, "ms": 0.0})
        e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    for r in csv.DictReader(open(glob.glob(os.path.join(d, "*kernel_trace.csv"))[0])):
        k = int(r["Dispatch_Id"])
        if k in out:
            out[k]["ms"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    return out


def build_counter_table(fetch_dir: str, write_dir: str, sq_dir: str) -> str:
    """Markdown rows: every kernel of the second FP64 build of --profile-build
    (from its FP64 sketch launch to the 1 GiB copy's fill), HBM bytes scaled by
    the copy as in traffic_summary, SQ instruction counts, counter-run times."""
    import re
    f, w, q = _load_pmc(fetch_dir), _load_pmc(write_dir), _load_pmc(sq_dir)
    gib_kib = float(1 << 20)
    # the 1 GiB copy is the largest copy of the run
    fs = gib_kib / max(v["c"].get("FETCH_SIZE", 0.0) for v in f.values() if "copyBuffer" in v["name"])
    ws = gib_kib / max(v["c"].get("WRITE_SIZE", 0.0) for v in w.values() if "copyBuffer" in v["name"])

    def short(name):
        m = re.search(r"::(\w+)(<[^>]*>)?\(", name)
        return (m.group(1) + (m.group(2) or "").replace(" ", "")) if m else name[:40]

    keys = sorted(f)
    sk = [k for k in keys if "sketch_f64" in f[k]["name"]]
    start = sk[1]
    end = next((k for k in keys if k > start and "FillFunctor" in f[k]["name"]), keys[-1] + 1)
    agg = {}
    for k in keys:
        if k < start or k >= end:
            continue
        a = agg.setdefault(short(f[k]["name"]), {"calls": 0, "ms": 0.0, "fetch": 0.0, "write": 0.0, "valu": 0.0,
                                                 "mfma": 0.0, "lds": 0.0})
        a["calls"] += 1
        a["fetch"] += f[k]["c"].get("FETCH_SIZE", 0.0) * fs * 1024
        a["write"] += w.get(k, {"c": {}})["c"].get("WRITE_SIZE", 0.0) * ws * 1024
        sq = q.get(k, {"c": {}, "ms": 0.0})
        a["valu"] += sq["c"].get("SQ_INSTS_VALU", 0.0)
        a["mfma"] += sq["c"].get("SQ_INSTS_MFMA", 0.0)
        a["lds"] += sq["c"].get("SQ_INSTS_LDS", 0.0)
        a["ms"] += sq["ms"]
    rows = [f"calibration: FETCH_SIZE x {fs:.3f}, WRITE_SIZE x {ws:.3f}", "",
            "| kernel | calls | ms | HBM fetch GB | HBM write GB | VALU instr | MFMA instr | LDS instr |",
            "|---|---|---|---|---|---|---|---|"]
    for n, a in sorted(agg.items(), key=lambda kv: -kv[1]["ms"]):
        rows.append(f"| `{n}` | {a['calls']} | {a['ms']:.3f} | {a['fetch'] / 1e9:.3f} | {a['write'] / 1e9:.3f} | "
                    f"{a['valu']:.3e} | {a['mfma']:.3e} | {a['lds']:.3e} |")
    return "\n".join(rows)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(w, sketch_passes: int, rows: int = 2048):
    """The oracle (plain NumPy FP64, never tuned) timed on this host.

    value: the oracle's time for the benchmarked 131072-point build, estimated
    from two bounded measurements on the same workload recipe, one thread:
      * its dense sketch of `rows` of the N rows x d0 columns, scaled to all
        rows and to the build's sketch passes (each pass evaluates all N^2
        kernel entries, which dominates the time);
      * everything else, from a full oracle build of the same recipe at
        n = 16384 minus that build's own sketch time, scaled by N / 16384 (the
        construction outside the sketch is O(n) in the paper's analysis).
    measured: full oracle builds of the 4096-point square with 1 and with all
    threads, and the 16384-point cube build above."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.build import build_h2
    from oracle.kernels import KernelOperator
    from oracle.philox import gaussian
    from paper_2506_16759_amd.workloads import SMALL_2D, uniform_points

    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()

    class TimedOperator(KernelOperator):
        """The oracle's kernel operator with its sketch time accumulated."""
        sketch_s = 0.0

        def sketch(self, omega):
            t0 = time.perf_counter()
            out = super().sketch(omega)
            self.sketch_s += time.perf_counter() - t0
            return out

    def full_build(pts, kind, length, wl, threads):
        op = TimedOperator(pts, kind, length)
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            h = build_h2(op, pts, wl.leaf_size, wl.eta, wl.tol, wl.d0, wl.d_inc, 256, wl.omega_seed)
            dt = time.perf_counter() - t0
        return dt, op.sketch_s, h.samples

    pts = w.points()
    op = KernelOperator(pts, w.kernel, w.length)
    omega = gaussian(w.omega_seed, np.arange(w.n), 0, w.d0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        op.sketch_rows(np.arange(rows), omega)
        t_rows = time.perf_counter() - t0
    sketch_est = t_rows * (w.n / rows) * sketch_passes
    n_mid = 16384
    p_mid = uniform_points(n_mid, w.dim, w.point_seed)
    t_mid1, s_mid1, samples_mid = full_build(p_mid, w.kernel, w.length, w, 1)
    rest_est = (t_mid1 - s_mid1) * (w.n / n_mid)
    s2 = SMALL_2D
    t_c0_1, _, _ = full_build(s2.points(), s2.kernel, s2.length, s2, 1)
    t_c0_n, _, _ = full_build(s2.points(), s2.kernel, s2.length, s2, nthreads)
    return {
        "value": sketch_est + rest_est,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one thread: the oracle's dense sketch of {rows} of {w.n} rows x {w.d0} columns ({t_rows:.2f} s) "
                   f"scaled to all rows and the build's {sketch_passes} sketch passes ({sketch_est:.0f} s), plus "
                   f"the rest of a full oracle build of the same recipe at n={n_mid} ({t_mid1 - s_mid1:.1f} s of "
                   f"{t_mid1:.1f} s, {samples_mid} samples) scaled by {w.n // n_mid} ({rest_est:.0f} s)"),
        "cpu": _cpu_model(),
        "host_threads": nthreads,
        "measured_full_builds_s": {
            f"{s2.name}_threads1": t_c0_1, f"{s2.name}_threads{nthreads}": t_c0_n,
            f"exp3d_n{n_mid}_threads1": t_mid1,
        },
    }


def bench_batched(h2, ctx, steps: int = 2):
    """The 64-problem covariance batch: leaf sizes and tile shapes from the
    autotuners, then batched FP64 and BF16X6 builds (one hipGraph each) against
    64 sequential single FP64 builds."""
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
        t0 = time.perf_counter()
        try:
            tuned = h2.autotune_tiles(ctx, probs, precision=prec, d_max=96)
        except h2.H2Error as exc:
            res[name] = {"error": str(exc)}
            continue
        tune_ms = (time.perf_counter() - t0) * 1e3
        print(f"[bench] batched {name} tiles {tuned['sketch_cols']}/{tuned['bsr_cols']} "
              f"({', '.join(f'{v:.1f}' for v in tuned['times_ms'])} ms)", file=sys.stderr, flush=True)
        for i in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                mats, info = h2.build_batched(ctx, probs, precision=prec, d_max=96, return_info=True,
                                              sketch_cols=tuned["sketch_cols"], bsr_cols=tuned["bsr_cols"])
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
                         "samples_range": [min(samples), max(samples)],
                         "tiles": {"sketch_cols": info["sketch_cols"], "bsr_cols": info["bsr_cols"],
                                   "tune_ms": tune_ms,
                                   "candidate_device_ms": dict(zip(
                                       ["sketch64", "sketch48", "sketch32", "bsr64", "bsr48", "bsr32", "bsr16"],
                                       tuned["times_ms"]))}}
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


def bench_scaling_series(h2, ctx, sizes=(1 << 15, 1 << 16, 1 << 17, 1 << 18)):
    """Doubling-N series of the FP64 build on the timed workload's recipe
    (uniform cube, exp(-r/0.2), leaf 64, eta 0.7, tol 1e-6): phase times,
    stored bytes and the device high-water mark per N (Sec. V-B: everything
    but the O(N^2) dense sketch grows linearly with N)."""
    import torch

    from paper_2506_16759_amd.workloads import CUBE_131K, uniform_points
    w = CUBE_131K
    out = []
    for n in sizes:
        pts = torch.from_numpy(uniform_points(n, w.dim, w.point_seed)).cuda()
        info = None
        for _ in range(2):   # the second build's numbers (pool pages mapped by the first)
            H = h2.build(ctx, pts, w.kernel, w.length, tol=w.tol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0,
                         d_inc=w.d_inc, seed=w.omega_seed)
            info = H.info()
            H.close()
        rec = {"n": n, "samples": info["samples"], "sketch_passes": info["sketch_calls"],
               "rank_range": [info["rank_min"], info["rank_max"]], "near_blocks": info["near_blocks"],
               "far_blocks": info["far_blocks"], "bytes_dense": info["bytes_dense"],
               "bytes_coupling": info["bytes_coupling"], "bytes_basis": info["bytes_basis"],
               "bytes_peak": info["bytes_peak"],
               "phases_ms": {k[2:]: round(info[k], 3) for k in info if k.startswith("t_")}}
        rec["non_sketch_ms"] = round(info["t_total"] - info["t_sample"], 3)
        out.append(rec)
        print(f"[bench] series n={n}: {info['t_total']:.1f} ms (sketch {info['t_sample']:.1f}), "
              f"peak {info['bytes_peak'] / 1e9:.2f} GB", file=sys.stderr, flush=True)
    return out


def _power_norm_ratio(apply_diff, apply_ref, n, iters=12, seed=7):
    """||A_diff||_2 / ||A_ref||_2 by power iteration on both symmetric operators
    (Sec. V-A measures the error this way against the sampler)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    norms = []
    for apply in (apply_diff, apply_ref):
        x = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        nrm = 0.0
        for _ in range(iters):
            x = x / torch.linalg.norm(x)
            x = apply(x)
            nrm = float(torch.linalg.norm(x))
        norms.append(nrm)
    return norms[0] / norms[1]


def bench_update_one(h2, ctx, n: int):
    """The rank-64 update workload at n points (child process): H's build, the
    update, their stored bytes and device high-water marks, and the error
    against the sampler on two vectors; an out-of-memory error is reported."""
    import torch

    from paper_2506_16759_amd.workloads import cube_update
    w = cube_update(n)
    b = w.base
    pts = torch.from_numpy(b.points()).cuda()
    rec = {"n": n, "rank": w.rank}
    try:
        H = h2.build(ctx, pts, b.kernel, b.length, tol=b.tol, leaf_size=b.leaf_size, eta=b.eta, d0=b.d0,
                     d_inc=b.d_inc, seed=b.omega_seed)
        hi = H.info()
        rec["old"] = {"ms": hi["t_total"], "samples": hi["samples"], "dense_gb": hi["bytes_dense"] / 1e9,
                      "coupling_gb": hi["bytes_coupling"] / 1e9, "peak_gb": hi["bytes_peak"] / 1e9}
        U, V = w.factors()
        Ut, Vt = torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Hu = h2.build_update(ctx, H, Ut, Vt, tol=w.tol, d0=w.d0, d_inc=w.d_inc, d_max=w.d_max, seed=w.omega_seed,
                             oversample=w.oversample)
        torch.cuda.synchronize()
        ui = Hu.info()
        x = torch.randn(2, n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5)).T
        ref = H.matvec(x) + Ut @ (Vt.T @ x)
        rec["update"] = {"ms": (time.perf_counter() - t0) * 1e3, "device_ms": ui["t_total"], "samples": ui["samples"],
                         "rank_range": [ui["rank_min"], ui["rank_max"]], "coupling_gb": ui["bytes_coupling"] / 1e9,
                         "basis_gb": ui["bytes_basis"] / 1e9, "peak_gb": ui["bytes_peak"] / 1e9,
                         "error_vs_sampler": float(torch.linalg.norm(Hu.matvec(x) - ref) / torch.linalg.norm(ref))}
    except h2.H2Error as exc:
        rec["error"] = str(exc)
    rec["device_total_gb"] = torch.cuda.get_device_properties(0).total_memory / 1e9
    return rec


def bench_update_series(sizes=(1 << 16, 1 << 17, 1 << 18, 1 << 19)):
    """The update workload at doubling sizes, each in a fresh process."""
    import subprocess
    out = []
    for n in sizes:
        cmd = [sys.executable, os.path.abspath(__file__), "--update-one", str(n)]
        res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        if res.returncode != 0:
            out.append({"n": n, "error": f"exit {res.returncode}: {res.stderr[-500:]}"})
        else:
            out.append(json.loads(res.stdout.strip().splitlines()[-1]))
        print(f"[bench] update series n={n}: {json.dumps(out[-1])[:300]}", file=sys.stderr, flush=True)
    return out


TABLE2_PROBLEMS = {"covariance": ("covariance exp(-r/0.2)", "exp", 0.2),
                   "helmholtz": ("helmholtz cos(3r)/r", "helmholtz", 3.0)}


def bench_table2_one(h2, ctx, problem: str, leaf: int, mode: str, n=1 << 18):
    """One configuration of Table II's setting: the black box is the product
    with an existing H^2 matrix (Sec. V-A), entries come from the kernel,
    N = 2^18 uniform points in the cube, tol 1e-6; fixed sample size d = leaf
    size (Sec. III-A, no convergence test) or adaptive sampling with blocks of
    32 columns (Sec. III-B).  The black-box matrix is this library's own H^2
    matrix of the kernel built from the dense sketch at tol 1e-8, leaf 64.
    Error: relative 2-norm distance to the black box by power iteration."""
    import torch

    from paper_2506_16759_amd.workloads import uniform_points
    prob, kind, par = TABLE2_PROBLEMS[problem]
    kw = dict(wavenumber=par) if kind == "helmholtz" else dict(length=par)
    pts = torch.from_numpy(uniform_points(n, 3, 1)).cuda()
    t0 = time.perf_counter()
    Hbb = h2.build(ctx, pts, kind, tol=1e-8, leaf_size=64, **kw)
    bb_ms = (time.perf_counter() - t0) * 1e3
    d0, dinc = (leaf, 0) if mode == "fixed" else (32, 32)
    # three builds; the faster of the last two is reported (the first maps the
    # memory, and right after another process released its ~180 GB a build can
    # spend seconds mapping its ~100 GB of dense blocks), all times listed
    times, infos, H, best = [], [], None, None
    for rep in range(3):
        if H is not None:
            H.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = h2.build(ctx, pts, kind, sketch=Hbb, tol=1e-6, leaf_size=leaf, d0=d0, d_inc=dinc, d_max=256, seed=1001,
                     **kw)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        infos.append(H.info())
    best = 1 if times[1] <= times[2] else 2
    info = infos[best]
    err = _power_norm_ratio(lambda x: H.matvec(x) - Hbb.matvec(x), Hbb.matvec, n)
    stored = info["bytes_dense"] + info["bytes_coupling"] + info["bytes_basis"]
    return {"problem": prob, "mode": mode, "leaf": leaf, "sample_block": d0 if mode == "fixed" else 32,
            "total_samples": info["samples"], "build_ms": times[best], "all_build_ms": times,
            "device_ms": info["t_total"],
            "rank_range": [info["rank_min"], info["rank_max"]], "stored_gb": stored / 1e9,
            "peak_gb": info["bytes_peak"] / 1e9, "rel_error_2norm": err, "sketch_calls": info["sketch_calls"],
            "black_box": {"samples": Hbb.info()["samples"], "build_ms": bb_ms},
            "phases_ms": {k[2:]: round(info[k], 3) for k in info if k.startswith("t_")}}


def bench_table2():
    """Every configuration of Table II's setting, each in a fresh process: a
    ~100 GB matrix next to the ~80 GB black box leaves the memory pools in a
    state that depends on the previous builds, so every configuration starts
    from a clean device (the first of its two builds maps the memory)."""
    import subprocess
    rows = []
    for problem in TABLE2_PROBLEMS:
        for leaf in (256, 128):
            for mode in ("fixed", "adaptive"):
                cmd = [sys.executable, os.path.abspath(__file__), "--table2-one", f"{problem},{leaf},{mode}"]
                res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
                if res.returncode != 0:
                    raise RuntimeError(f"{' '.join(cmd)} failed ({res.returncode}):\n{res.stderr[-2000:]}")
                rec = json.loads(res.stdout.strip().splitlines()[-1])
                rows.append(rec)
                print(f"[bench] table2 {rec['problem']} leaf {leaf} {mode}: {rec['build_ms']:.1f} ms, samples "
                      f"{rec['total_samples']}, ranks {rec['rank_range'][0]}..{rec['rank_range'][1]}, "
                      f"{rec['stored_gb']:.2f} GB, error {rec['rel_error_2norm']:.3e}", file=sys.stderr, flush=True)
    return rows


def first_pass_columns(h2, w) -> int:
    """Columns of a build's first sketch pass: d0 plus the default look-ahead."""
    o = h2.opts_default()
    return min(w.d0 + o.sketch_ahead, o.d_max)


def load_goldens() -> dict:
    """The oracle's stored results for the benchmarked cube (written by
    tests/golden/make_cube_golden.py, which runs only the oracle), by tol."""
    out = {}
    gdir = os.path.join(ROOT, "tests", "golden")
    for name in sorted(os.listdir(gdir)):
        if name.startswith("cube_exp3d_n131072_tol") and name.endswith(".json"):
            g = json.load(open(os.path.join(gdir, name)))
            out[float(g["tol"])] = g
    return out


def sampled_errors(H, golden: dict, tol: float) -> dict:
    """Relative error of the built matrix's product on the stored sampled rows:
    against the exact kernel rows, and against the FP64 oracle's H^2 matrix
    built at the same tolerance (when the oracle's result is stored)."""
    import numpy as np
    import torch

    from paper_2506_16759_amd.workloads import gaussian_vectors
    if not golden:
        return {}
    g0 = next(iter(golden.values()))
    rows = np.array(g0["rows"])
    x = gaussian_vectors(g0["n"], 4, g0["x_seed"])
    xt = torch.from_numpy(np.ascontiguousarray(x.T)).cuda().T
    y = H.matvec(xt).cpu().numpy()[rows]
    y_exact = np.array(g0["y_exact"])
    out = {"rows": len(rows), "vs_exact": float(np.linalg.norm(y - y_exact) / np.linalg.norm(y_exact))}
    g = golden.get(float(tol))
    if g is not None:
        y_or = np.array(g["y_h2"])
        out["vs_fp64_oracle"] = float(np.linalg.norm(y - y_or) / np.linalg.norm(y_or))
        out["oracle_samples"] = g["samples"]
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
    ap.add_argument("--scaling-series", action="store_true",
                    help="only the doubling-N series of the FP64 build (2^15..2^18 points), one JSON line")
    ap.add_argument("--table2", action="store_true",
                    help="only the fixed-vs-adaptive runs of Table II's setting (2^18 points, H^2 black box)")
    ap.add_argument("--table2-one", default=None, help=argparse.SUPPRESS)   # problem,leaf,mode (child process)
    ap.add_argument("--update-series", action="store_true",
                    help="only the rank-64 update workload at 2^16..2^19 points (time, memory), one JSON line")
    ap.add_argument("--update-one", type=int, default=0, help=argparse.SUPPRESS)   # n (child process)
    ap.add_argument("--profile-build", action="store_true",
                    help="only two FP64 builds of the benchmarked cube and a 1 GiB copy of known size, for counter "
                         "collection on every kernel of a build")
    ap.add_argument("--traffic-from", default=None,
                    help="FETCH_DIR,WRITE_DIR[,SQ_DIR]: rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (/ SQ counter) output "
                         "directories of --profile-kernels; write the sketch launches' HBM bytes (scaled by the 1 GiB "
                         "copy, with the SQ counters if given) as JSON to stdout")
    ap.add_argument("--build-counters", default=None,
                    help="FETCH_DIR,WRITE_DIR,SQ_DIR: rocprofv3 --pmc output directories of --profile-build; print "
                         "the per-kernel counter table of its second build (markdown rows)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only run the sketch (FP64, FP32, bf16x3, FP32E, bf16x6, FP64_SYM; the first pass's 64 columns) "
                         "twice each and a 1 GiB copy of known size, for counter collection")
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(traffic_summary(*args.traffic_from.split(",")), indent=1))
        return
    if args.build_counters:
        print(build_counter_table(*args.build_counters.split(",")))
        return
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
        nc = first_pass_columns(h2, w)
        omega = h2.gaussian(ctx, w.omega_seed, torch.arange(w.n, dtype=torch.int32), 0, nc)
        for prec in (h2.FP64, h2.FP32, h2.BF16X3, h2.FP32E, h2.BF16X6, h2.FP64_SYM):
            for _ in range(2):
                h2.sketch(ctx, pts, w.kernel, w.length, omega, precision=prec)
        # calibration: a plain device copy of exactly 1 GiB (reads 1 GiB, writes 1 GiB)
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_kernels": "done", "copy_bytes": a.numel() * 8}), flush=True)
        return
    if args.scaling_series:
        print(json.dumps({"scaling_series": bench_scaling_series(h2, h2.Context(0))}), flush=True)
        return
    if args.table2:
        print(json.dumps({"table2": bench_table2()}), flush=True)
        return
    if args.update_series:
        print(json.dumps({"update_series": bench_update_series()}), flush=True)
        return
    if args.update_one:
        print(json.dumps(bench_update_one(h2, h2.Context(0), args.update_one)), flush=True)
        return
    if args.table2_one:
        problem, leaf, mode = args.table2_one.split(",")
        print(json.dumps(bench_table2_one(h2, h2.Context(0), problem, int(leaf), mode)), flush=True)
        return
    if args.profile_build:
        ctx = h2.Context(0)
        pts = torch.from_numpy(w.points()).cuda()
        for _ in range(2):
            H = h2.build(ctx, pts, w.kernel, w.length, tol=w.tol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0,
                         d_inc=w.d_inc, seed=w.omega_seed)
            H.close()
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_build": "done", "copy_bytes": a.numel() * 8}), flush=True)
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

    golden = load_goldens()

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
        ms = (time.perf_counter() - t0) / steps * 1e3
        # accuracy, outside the timed region, of one more build (the builds are
        # deterministic: it equals every timed one)
        H = h2.build(ctx, pts, w.kernel, w.length, opts=o)
        infos[-1]["errors"] = sampled_errors(H, golden, o.tol)
        H.close()
        return ms, times, infos[-1]

    ms_per_step, times, info = timed_builds(opts, "fp64", args.steps, args.warmup)

    # mixed precision on the same points at the same tolerance: three-term
    # split bf16 products (bf16x6), FP32 matrix cores (fp32), FP32 entries
    # contracted in FP64 (fp32e), FP64 with symmetric-tile reuse in the sketch
    # (fp64_sym); bf16x3 at tol 1e-4 (its products carry ~2^-17 relative
    # error), with FP64 at 1e-4 for comparison
    mixed = {}
    for name, prec, mtol in (("bf16x6", h2.BF16X6, tol), ("fp32", h2.FP32, tol), ("fp32e", h2.FP32E, tol),
                             ("fp64_sym", h2.FP64_SYM, tol),
                             ("fp64_tol1e-4", h2.FP64, 1e-4), ("bf16x3_tol1e-4", h2.BF16X3, 1e-4),
                             ("fp64_tol1e-8", h2.FP64, 1e-8), ("fp32e_tol1e-8", h2.FP32E, 1e-8)):
        o = h2.opts_default(tol=mtol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0, d_inc=w.d_inc, seed=w.omega_seed,
                            precision=prec)
        try:
            mms, mtimes, minfo = timed_builds(o, name, max(1, args.steps // 2 + 1), 1)
            mixed[name] = {"tol": mtol, "ms_per_build": mms, "samples": minfo["samples"],
                           "adaptive_rounds": minfo["rounds"], "rank_range": [minfo["rank_min"], minfo["rank_max"]],
                           "sketch_phase_ms": minfo["t_sample"], "sketch_passes": minfo["sketch_calls"],
                           "errors": minfo["errors"]}
            if mtol == tol:
                mixed[name]["speedup_vs_fp64"] = ms_per_step / mms
        except h2.H2Error as exc:
            mixed[name] = {"tol": mtol, "error": str(exc)}
    if "ms_per_build" in mixed.get("bf16x3_tol1e-4", {}) and "ms_per_build" in mixed.get("fp64_tol1e-4", {}):
        mixed["bf16x3_tol1e-4"]["speedup_vs_fp64"] = (mixed["fp64_tol1e-4"]["ms_per_build"]
                                                      / mixed["bf16x3_tol1e-4"]["ms_per_build"])

    # dominant kernel of the timed build: its one fused sketch pass (d0 plus
    # the look-ahead columns), timed live on the library's stream
    nc = first_pass_columns(h2, w)
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
    # and with symmetric-tile reuse (each entry of the upper block triangle
    # evaluated once; its timing includes the scratch reduction)
    h2.sketch(ctx, pts, w.kernel, w.length, omega, precision=h2.FP64_SYM)
    ev0.record(ctx.stream)
    for _ in range(args.sketch_launches):
        h2.sketch(ctx, pts, w.kernel, w.length, omega, precision=h2.FP64_SYM)
    ev1.record(ctx.stream)
    ev1.synchronize()
    sksym_ms = ev0.elapsed_time(ev1) / args.sketch_launches
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
        "sketch_fp64_sym_kernel_ms": sksym_ms,
        "mixed_vs_fp64_speedup": mixed.get("bf16x6", {}).get("speedup_vs_fp64"),
        "mixed": mixed,
        "samples": info["samples"],
        "sketch_passes": info["sketch_calls"],
        "errors": info["errors"],
        "adaptive_rounds": info["rounds"],
        "rank_range": [info["rank_min"], info["rank_max"]],
        "phases_ms": {k[2:]: round(info[k], 3) for k in info if k.startswith("t_")},
        "bytes": {"dense": info["bytes_dense"], "coupling": info["bytes_coupling"], "basis": info["bytes_basis"]},
        "roofline": {
            "kernel": f"sketch_f64_kernel<3,exp,{nc}>",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic(f"sketch_f64_kernel<3,exp,{nc}>"),
            "algorithmic_flop_per_launch": sketch_flops_per_entry(w.dim, nc) * entries,
            "launch_ms": sk_ms,
        },
    }
    if not args.no_extras:
        # the update first: its 27 GB of couplings would otherwise wait for the
        # memory pool to map new pages past what the batched builds left cached
        out["update"] = bench_update(h2, ctx)
        out["batched"] = bench_batched(h2, ctx)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        passes = 1 + max(0, info["samples"] - w.d0) // w.d_inc   # the oracle draws d_inc columns per round
        out["cpu_baseline"] = cpu_baseline(w, passes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
