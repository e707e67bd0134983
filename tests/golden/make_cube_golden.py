"""Writes the oracle's construction of the 131072-point covariance cube.

    python tests/golden/make_cube_golden.py [tol ...]      (default: 1e-6 1e-8)

Runs only the oracle (Alg. 1 with the adaptive sampling of Sec. III-B, FP64)
on the seeded 131072-point cube (exp(-r/0.2), leaf 64, eta 0.7, d0 32, +16 per
round, Omega seed 1001) and stores what a GPU test of the full-size workload
compares with: the sample count, rounds per depth, threshold, top depth, the
ranks of every processed cluster, a SHA-256 of each depth's skeleton indices
(original point order, node by node, int32 little-endian: the layout of the
library's SKEL export), and the products of the oracle's H^2 matrix and of the
exact kernel with four seeded vectors on 64 seeded rows.  The oracle's wall
time on the machine that ran it is recorded as information.  The dense sketch
makes this an O(N^2) run of tens of minutes per tolerance.
"""
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.build import build_h2  # noqa: E402
from oracle.kernels import KernelOperator  # noqa: E402
from paper_2506_16759_amd.workloads import CUBE_131K, gaussian_vectors  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def golden_path(tol: float) -> str:
    return os.path.join(HERE, f"cube_exp3d_n131072_tol{tol:.0e}.json")


def main(tols):
    w = CUBE_131K
    pts = w.points()
    op = KernelOperator(pts, w.kernel, w.length)
    x = gaussian_vectors(w.n, 4, 31)
    rows = np.sort(np.random.default_rng(32).choice(w.n, 64, replace=False))
    y_exact = op.entries(rows, np.arange(w.n)) @ x
    for tol in tols:
        t0 = time.perf_counter()
        h = build_h2(op, pts, w.leaf_size, w.eta, tol, w.d0, w.d_inc, 256, w.omega_seed)
        dt = time.perf_counter() - t0
        D = h.tree.depth
        perm = h.tree.perm
        ranks, skel_sha = {}, {}
        for t in range(h.top, D + 1):
            ranks[str(t)] = [h.rank(t, i) for i in range(1 << t)]
            sk = np.concatenate([perm[np.asarray(h.skel[(t, i)], dtype=np.int64)] for i in range(1 << t)])
            skel_sha[str(t)] = hashlib.sha256(sk.astype("<i4").tobytes()).hexdigest()
        y_h2 = h.matvec(x)[rows]
        out = {
            "source": "oracle: build_h2 (Alg. 1 + Sec. III-B, FP64)",
            "workload": w.name, "n": w.n, "dim": w.dim, "kernel": w.kernel, "length": w.length,
            "leaf_size": w.leaf_size, "eta": w.eta, "tol": tol, "d0": w.d0, "d_inc": w.d_inc, "d_max": 256,
            "omega_seed": w.omega_seed,
            "samples": h.samples, "rounds": {str(k): v for k, v in h.rounds.items()}, "delta": h.delta,
            "top": h.top, "ranks": ranks, "skel_sha256": skel_sha,
            "x_seed": 31, "rows_seed": 32, "rows": rows.tolist(),
            "y_h2": y_h2.tolist(), "y_exact": y_exact.tolist(),
            "oracle_seconds": dt, "oracle_host": f"{platform.processor() or platform.machine()}, "
                                                 f"{os.cpu_count()} logical CPUs",
        }
        with open(golden_path(tol), "w") as f:
            json.dump(out, f)
        err = np.linalg.norm(y_h2 - y_exact) / np.linalg.norm(y_exact)
        print(f"tol {tol:g}: samples {h.samples}, ranks {min(min(r) for r in ranks.values())}.."
              f"{max(max(r) for r in ranks.values())}, sampled-row error {err:.3e}, oracle {dt:.0f} s",
              flush=True)
        del h


if __name__ == "__main__":
    main([float(a) for a in sys.argv[1:]] or [1e-6, 1e-8])
