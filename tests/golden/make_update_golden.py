"""Writes the oracle's result for the low-rank update workload at n = 2^14.

    python tests/golden/make_update_golden.py

Runs only the oracle (the symmetric construction of H, then the two-sided
construction of H + U V^T, Alg. 1 + Sec. III-B) on the seeded inputs of
``cube_update(16384)`` and stores what a GPU test can compare with: sample
counts, ranks per depth on both sides, the threshold, and the products of the
oracle's update and of H + U V^T with two seeded vectors on 64 seeded rows.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.build import build_h2  # noqa: E402
from oracle.kernels import KernelOperator  # noqa: E402
from oracle.update import update_h2  # noqa: E402
from paper_2506_16759_amd.workloads import cube_update, gaussian_vectors  # noqa: E402


def main():
    w = cube_update(1 << 14)
    b = w.base
    pts = b.points()
    h = build_h2(KernelOperator(pts, b.kernel, b.length), pts, b.leaf_size, b.eta, b.tol, b.d0, b.d_inc, 128,
                 b.omega_seed)
    U, V = w.factors()
    hu = update_h2(h, pts, U, V, b.leaf_size, b.eta, w.tol, w.d0, w.d_inc, w.d_max, w.omega_seed,
                   oversample=w.oversample)
    x = gaussian_vectors(w.n, 2, 21)
    rows = np.sort(np.random.default_rng(22).choice(w.n, 64, replace=False))
    y_upd = hu.matvec(x)[rows]
    y_ref = (h.matvec(x) + U @ (V.T @ x))[rows]
    D = hu.tree.depth
    out = {
        "source": "oracle: build_h2 then update_h2 (Alg. 1 + Sec. III-B, two-sided)",
        "workload": w.name, "n": w.n, "rank": w.rank, "tol": w.tol,
        "old_samples": h.samples, "samples": hu.samples, "top": hu.top, "delta": hu.delta,
        "ranks": {str(t): [hu.rank(t, i) for i in range(1 << t)] for t in range(hu.top, D + 1)},
        "ranks_c": {str(t): [hu.rank_c(t, i) for i in range(1 << t)] for t in range(hu.top, D + 1)},
        "x_seed": 21, "rows_seed": 22, "rows": rows.tolist(),
        "y_update": y_upd.tolist(), "y_reference": y_ref.tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "update_exp3d_n16384_r64.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, "samples", h.samples, hu.samples)


if __name__ == "__main__":
    main()
