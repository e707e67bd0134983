"""Batched construction (many independent problems in one launch sequence).

The batched path runs the same kernels as single builds over concatenated
problems, sketches the first launch sequence's columns up front (problems not
converged within them are built again with d_max columns) and picks each
problem's column count with a prefix QR per cluster.  It must therefore
reproduce, problem by problem, what a single build with the same d_max and a
look-ahead of d_max - d0 columns computes:
  * tree, lists and top depth bit-exact (same host plan),
  * the same sample count and the same ranks (the thresholds agree to 1e-12;
    the norm estimate is summed in another order),
  * matvec within the accuracy bound of each other and of the exact kernel.
Every problem of the batch is also compared with the oracle's construction of
the same problem: in FP64 the same sample count, threshold, ranks and
skeletons, blocks to entry rounding and ID matrices within the conditioning
bar of tests/gpu_util.py; in FP32 and BF16X6 the product error against the
oracle's matrix is stated and held to the accuracy bound.
Graph and eager launches of the batch run identical kernels: bit-identical.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_16759_amd as h2
from paper_2506_16759_amd.workloads import batch_problems, uniform_points
from oracle.build import build_h2
from oracle.kernels import KernelOperator
from gpu_util import compare_with_oracle



def _say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return h2.Context(0)


def _np(t):
    return t.detach().cpu().numpy()


def _colmajor_from(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).cuda().T


# (n, dim, kernel, length, leaf, tol, d0, d_inc, seed); includes a problem with
# no admissible block, a 1-D problem, ragged leaves and a problem needing rounds
MIXED_BATCH = [
    (5000, 3, "exp", 0.2, 64, 1e-6, 32, 16, 1),
    (50, 2, "exp", 0.2, 64, 1e-6, 32, 16, 2),
    (3333, 2, "gauss", 0.1, 40, 1e-6, 32, 16, 3),
    (2100, 1, "exp", 0.3, 32, 1e-8, 16, 8, 4),
    (6000, 3, "exp", 0.2, 64, 1e-7, 16, 16, 5),
    (777, 3, "gauss", 0.15, 24, 1e-6, 32, 16, 6),
]


def _problems(spec):
    out = []
    for i, (n, dim, kind, length, leaf, tol, d0, dinc, seed) in enumerate(spec):
        out.append(dict(points=uniform_points(n, dim, 300 + i), kernel=kind, length=length, leaf_size=leaf,
                        tol=tol, eta=0.7, d0=d0, d_inc=dinc, seed=seed))
    return out


def _factors(H):
    D, top = int(H.export("DEPTH")[0]), int(H.export("TOP")[0])
    return dict(ranks=[H.export("RANKS", t) for t in range(top, D + 1)],
                skel=[H.export("SKEL", t) for t in range(top, D + 1)],
                basis=[H.export("BASIS", t) for t in range(top, D + 1)],
                coupling=[H.export("COUPLING", t) for t in range(top, D + 1)],
                dense=H.export("DENSE"))


def test_batched_matches_single_builds(ctx):
    probs = _problems(MIXED_BATCH)
    dmax = 96
    _say(f"batched vs single: {len(probs)} problems, n={[p['points'].shape[1] for p in probs]}, d_max={dmax}")
    mats, info = h2.build_batched(ctx, probs, d_max=dmax, use_graph=True, return_info=True)
    _say(f"batch info {info}")
    for i, (p, Hb) in enumerate(zip(probs, mats)):
        n = p["points"].shape[1]
        _say(f"problem {i}: n={n} single build")
        Hs = h2.build(ctx, p["points"], p["kernel"], p["length"], tol=p["tol"], leaf_size=p["leaf_size"],
                      eta=p["eta"], d0=p["d0"], d_inc=p["d_inc"], seed=p["seed"], d_max=dmax,
                      sketch_ahead=dmax - p["d0"])
        for part in ("DEPTH", "PERM", "NODES", "NEAR_PTR", "NEAR_IDX", "TOP"):
            np.testing.assert_array_equal(Hb.export(part), Hs.export(part))
        D = int(Hs.export("DEPTH")[0])
        for t in range(D + 1):
            np.testing.assert_array_equal(Hb.export("FAR_PTR", t), Hs.export("FAR_PTR", t))
            np.testing.assert_array_equal(Hb.export("FAR_IDX", t), Hs.export("FAR_IDX", t))
        ib, is_ = Hb.info(), Hs.info()
        np.testing.assert_allclose(Hb.export("DENSE"), Hs.export("DENSE"), rtol=1e-14, atol=0)
        top = int(Hs.export("TOP")[0])
        if top <= D:
            assert abs(ib["delta"] - is_["delta"]) <= 1e-12 * is_["delta"]
            assert ib["samples"] == is_["samples"], (ib["samples"], is_["samples"])
            fb, fs = _factors(Hb), _factors(Hs)
            diff = sum(int((a != b).sum()) for a, b in zip(fb["ranks"], fs["ranks"]))
            total = sum(a.size for a in fs["ranks"])
            _say(f"problem {i}: samples={ib['samples']} ranks {ib['rank_min']}..{ib['rank_max']}, "
                 f"{diff}/{total} ranks differ")
            assert diff == 0
        K = KernelOperator(p["points"], p["kernel"], p["length"]).dense()
        x = np.random.default_rng(i).standard_normal((n, 4))
        yb = _np(Hb.matvec(_colmajor_from(x)))
        ys = _np(Hs.matvec(_colmajor_from(x)))
        kx = K @ x
        eb = np.linalg.norm(yb - kx) / np.linalg.norm(kx)
        es = np.linalg.norm(yb - ys) / np.linalg.norm(kx)
        _say(f"problem {i}: matvec error vs K {eb:.3e}, vs single build {es:.3e}")
        assert eb <= 10 * p["tol"] and es <= 10 * p["tol"]
        Hs.close()
    for H in mats:
        H.close()


def test_batched_matches_oracle(ctx):
    """Every problem of a mixed batch against the oracle's construction of the
    same problem (Alg. 1 with adaptive sampling, d_inc columns at a time):
    FP64 gives the same sample count, threshold, ranks and skeletons, blocks to
    entry rounding and ID matrices to the ID conditioning; the FP32 and BF16X6
    batches state their product error against the oracle's matrix and keep the
    accuracy bound against the exact kernel."""
    probs = _problems(MIXED_BATCH)
    dmax = 96
    _say(f"batched vs oracle: n={[p['points'].shape[1] for p in probs]}")
    oracle = []
    for i, p in enumerate(probs):
        n = p["points"].shape[1]
        op = KernelOperator(p["points"], p["kernel"], p["length"])
        ho = build_h2(op, p["points"], p["leaf_size"], p["eta"], p["tol"], p["d0"], p["d_inc"], dmax, p["seed"])
        oracle.append((op, ho))
    mats = h2.build_batched(ctx, probs, d_max=dmax)
    for i, (p, H, (op, ho)) in enumerate(zip(probs, mats, oracle)):
        info = H.info()
        _say(f"problem {i}: n={p['points'].shape[1]} samples {info['samples']} (oracle {ho.samples}) "
             f"ranks {info['rank_min']}..{info['rank_max']}")
        if ho.top <= ho.tree.depth:
            assert info["samples"] == ho.samples
            assert abs(info["delta"] - ho.delta) <= 1e-12 * ho.delta
        diff = compare_with_oracle(H, ho)
        _say(f"problem {i}: ID matrix differences {diff}")
    # the reduced-precision sketches carry ~1e-7 relative entry error: their
    # batches hold the problems at tol >= 1e-6
    keep = [i for i, p in enumerate(probs) if p["tol"] >= 1e-6]
    for prec, name in ((h2.FP64, "fp64"), (h2.FP32, "fp32"), (h2.BF16X6, "bf16x6")):
        sel = list(range(len(probs))) if prec == h2.FP64 else keep
        ms = mats if prec == h2.FP64 else h2.build_batched(ctx, [probs[i] for i in keep], precision=prec,
                                                             d_max=dmax)
        for i, H in zip(sel, ms):
            p, (op, ho) = probs[i], oracle[i]
            n = p["points"].shape[1]
            x = np.random.default_rng(40 + i).standard_normal((n, 3))
            y = _np(H.matvec(_colmajor_from(x)))
            yo, kx = ho.matvec(x), op.sketch(x)
            e_or = np.linalg.norm(y - yo) / np.linalg.norm(yo)
            e_k = np.linalg.norm(y - kx) / np.linalg.norm(kx)
            _say(f"{name} problem {i}: error vs oracle {e_or:.3e}, vs exact {e_k:.3e}, "
                 f"samples {H.info()['samples']} (oracle {ho.samples})")
            assert e_k <= 10 * p["tol"]
            if prec == h2.FP64:
                assert e_or <= 1e-10
            else:
                assert e_or <= 10 * p["tol"]
        for H in ms:
            H.close()


def test_batched_graph_equals_eager(ctx):
    probs = _problems(MIXED_BATCH[:4])
    _say("batched graph vs eager launch")
    mg, ig = h2.build_batched(ctx, probs, d_max=64, use_graph=True, return_info=True)
    me, ie = h2.build_batched(ctx, probs, d_max=64, use_graph=False, return_info=True)
    _say(f"graph nodes {ig['graph_nodes']}, device ms graph {ig['t_device_ms']:.2f} eager {ie['t_device_ms']:.2f}")
    assert ig["graph_nodes"] > 0 and ie["graph_nodes"] == 0
    for a, b in zip(mg, me):
        assert a.info()["samples"] == b.info()["samples"]
        fa, fb = _factors(a), _factors(b)
        for key in ("ranks", "skel", "basis", "coupling"):
            for u, v in zip(fa[key], fb[key]):
                np.testing.assert_array_equal(u, v)
        np.testing.assert_array_equal(fa["dense"], fb["dense"])


def test_batched_graph_replays_are_identical(ctx):
    """Two batched builds of the same problems (each capturing and launching its
    own graph, with eager work in between) give identical factors."""
    import torch
    probs = _problems(MIXED_BATCH[2:5])
    _say("batched graph repeat")
    m1 = h2.build_batched(ctx, probs, d_max=64)
    torch.ones(1 << 20, device="cuda").sum().item()
    m2 = h2.build_batched(ctx, probs, d_max=64)
    for a, b in zip(m1, m2):
        fa, fb = _factors(a), _factors(b)
        for key in ("ranks", "skel", "basis", "coupling"):
            for u, v in zip(fa[key], fb[key]):
                np.testing.assert_array_equal(u, v)


def test_batched_second_pass_equals_one_pass(ctx):
    """Problems not converged within the first launch sequence's columns are
    built again with d_max columns; every problem's construction equals that of
    one sequence with d_max columns (Omega is counter-based, the prefix test at
    a count ignores later columns, problems are independent): the same sample
    counts, ranks and skeletons, and factors to rounding (the ID kernel is
    chosen by the sequence's column capacity, so the two sequences may sum in
    different orders)."""
    probs = _problems(MIXED_BATCH)
    _say("batched: first pass of 32 columns + second pass vs one pass of 96")
    m1, i1 = h2.build_batched(ctx, probs, d_max=96, first_pass=96, return_info=True)
    m2, i2 = h2.build_batched(ctx, probs, d_max=96, first_pass=32, return_info=True)
    _say(f"one pass: first {i1['first_pass']} rerun {i1['second_pass']}; "
         f"two passes: first {i2['first_pass']} rerun {i2['second_pass']}")
    assert i1["first_pass"] == 96 and i1["second_pass"] == 0
    assert i2["first_pass"] == 32 and 0 < i2["second_pass"] < len(probs)
    for a, b in zip(m1, m2):
        assert a.info()["samples"] == b.info()["samples"]
        fa, fb = _factors(a), _factors(b)
        for key in ("ranks", "skel"):
            for u, v in zip(fa[key], fb[key]):
                np.testing.assert_array_equal(u, v)
        for key in ("basis", "coupling"):
            for u, v in zip(fa[key], fb[key]):
                np.testing.assert_allclose(u, v, rtol=0, atol=1e-9 * max(np.abs(v).max(initial=0.0), 1e-300))
        np.testing.assert_array_equal(fa["dense"], fb["dense"])
    for H in m1 + m2:
        H.close()


def test_batched_sample_limit_is_reported(ctx):
    _say("batched error path: d_max reached")
    probs = _problems([(3000, 3, "exp", 0.2, 48, 1e-10, 8, 8, 6), (2000, 2, "exp", 0.2, 64, 1e-6, 8, 8, 7)])
    with pytest.raises(h2.H2Error) as ei:
        h2.build_batched(ctx, probs, d_max=16)
    assert ei.value.status == -5


@pytest.mark.parametrize("precision,tol", [(1, 1e-6), (1, 1e-4), (2, 1e-4), (4, 1e-6)])
def test_batched_mixed_precision_meets_tol(ctx, precision, tol):
    spec = [(4000, 3, "exp", 0.2, 64, tol, 32, 16, 8), (2500, 2, "gauss", 0.1, 64, tol, 32, 16, 9)]
    probs = _problems(spec)
    _say(f"batched precision={precision} tol={tol}")
    mats = h2.build_batched(ctx, probs, precision=precision, d_max=96)
    for p, H in zip(probs, mats):
        n = p["points"].shape[1]
        K = KernelOperator(p["points"], p["kernel"], p["length"]).dense()
        x = np.random.default_rng(n).standard_normal((n, 4))
        y = _np(H.matvec(_colmajor_from(x)))
        e = np.linalg.norm(y - K @ x) / np.linalg.norm(K @ x)
        _say(f"n={n} samples={H.info()['samples']} matvec error {e:.3e}")
        assert e <= 10 * tol


def test_batched_covariance_workload_sampled(ctx):
    """The 64-problem covariance batch at full sizes: sampled matvec rows of
    every 8th problem against the exact kernel rows."""
    ws = batch_problems()
    _say(f"64-problem batch, total n={sum(w.n for w in ws)}")
    probs = [dict(points=w.points(), kernel=w.kernel, length=w.length, leaf_size=w.leaf_size, tol=w.tol,
                  eta=w.eta, d0=w.d0, d_inc=w.d_inc, seed=w.omega_seed) for w in ws]
    mats, info = h2.build_batched(ctx, probs, d_max=96, return_info=True)
    _say(f"batch info {info}")
    for i in range(0, len(ws), 8):
        w, H = ws[i], mats[i]
        op = KernelOperator(probs[i]["points"], w.kernel, w.length)
        rows = np.random.default_rng(i).choice(w.n, 32, replace=False)
        x = np.random.default_rng(100 + i).standard_normal((w.n, 2))
        y = _np(H.matvec(_colmajor_from(x)))
        kx = op.entries(rows, np.arange(w.n)) @ x
        e = np.linalg.norm(y[rows] - kx) / np.linalg.norm(kx)
        _say(f"problem {i}: n={w.n} dim={w.dim} {w.kernel} l={w.length:.3f} samples={H.info()['samples']} "
             f"sampled matvec error {e:.3e}")
        assert e <= 10 * w.tol
    for H in mats:
        H.close()


def test_autotuned_leaf_sizes(ctx):
    """The autotuner returns one of the candidates for every problem, the same
    one within a (dim, kernel, log2 n) group, and the tuned batch is accurate."""
    ws = batch_problems(count=10, seed=11)
    probs = [dict(points=w.points(), kernel=w.kernel, length=w.length, tol=w.tol, eta=w.eta, d0=w.d0,
                  d_inc=w.d_inc, seed=w.omega_seed) for w in ws]
    _say(f"autotune leaf sizes for n={[w.n for w in ws]}")
    leaves = h2.autotune_leaf(ctx, probs, candidates=(32, 64, 128), d_max=96)
    _say(f"tuned leaves {leaves}")
    assert all(l in (32, 64, 128) for l in leaves)
    groups = {}
    for w, l in zip(ws, leaves):
        groups.setdefault((w.dim, w.kernel, int(np.floor(np.log2(w.n)))), set()).add(l)
    assert all(len(v) == 1 for v in groups.values())
    for p, l in zip(probs, leaves):
        p["leaf_size"] = l
    mats = h2.build_batched(ctx, probs, d_max=96)
    for w, p, H in zip(ws, probs, mats):
        op = KernelOperator(p["points"], w.kernel, w.length)
        rows = np.random.default_rng(w.n).choice(w.n, 16, replace=False)
        x = np.random.default_rng(1).standard_normal((w.n, 2))
        y = _np(H.matvec(_colmajor_from(x)))
        kx = op.entries(rows, np.arange(w.n)) @ x
        assert np.linalg.norm(y[rows] - kx) / np.linalg.norm(kx) <= 10 * w.tol
        H.close()


def _same_factors(a, b):
    for key in ("ranks", "skel", "basis", "coupling"):
        for x, y in zip(a[key], b[key]):
            assert np.array_equal(x, y), key
    assert np.array_equal(a["dense"], b["dense"])


@pytest.mark.parametrize("precision", ["fp64", "bf16x6"])
def test_tile_shapes_give_identical_matrices(ctx, precision):
    """Every tile shape of the batched launches (columns per sketch launch,
    column-tile width of the block-sparse products) gives the same matrices
    bit for bit: each column's sums run in the same order whatever the tile."""
    # the split-bf16 sketch stops at FP32-level accuracy: problems at tol >= 1e-6
    probs = _problems([q for q in MIXED_BATCH if precision == "fp64" or q[5] >= 1e-6])
    _say(f"tile shapes {precision}")
    ref_mats, ref_info = h2.build_batched(ctx, probs, precision=precision, d_max=96, return_info=True)
    assert (ref_info["sketch_cols"], ref_info["bsr_cols"]) == (64, 64)
    ref = [_factors(H) for H in ref_mats]
    for H in ref_mats:
        H.close()
    for sk, bc in ((16, 64), (32, 16), (48, 48), (64, 32), (32, 48)):
        _say(f"tile shapes {precision} sketch_cols={sk} bsr_cols={bc}")
        mats, info = h2.build_batched(ctx, probs, precision=precision, d_max=96, return_info=True,
                                      sketch_cols=sk, bsr_cols=bc)
        assert (info["sketch_cols"], info["bsr_cols"]) == (sk, bc)
        for H, r in zip(mats, ref):
            _same_factors(_factors(H), r)
            H.close()


def test_autotuned_tile_shapes(ctx):
    """The tile autotuner times every candidate, returns the fastest it saw,
    and the batch built with the tuned shapes is the default batch bit for bit."""
    probs = _problems(MIXED_BATCH[:4])
    _say("autotune tile shapes")
    tuned = h2.autotune_tiles(ctx, probs, d_max=96)
    _say(f"tuned {tuned}")
    t = tuned["times_ms"]
    assert all(v > 0 for v in t)
    sk, bc = tuned["sketch_cols"], tuned["bsr_cols"]
    assert sk in (64, 48, 32) and bc in (64, 48, 32, 16)
    assert t[(64, 48, 32).index(sk)] == min(t[:3])
    assert t[3 + (64, 48, 32, 16).index(bc)] == min(t[3:])
    ref = h2.build_batched(ctx, probs, d_max=96)
    mats = h2.build_batched(ctx, probs, d_max=96, sketch_cols=sk, bsr_cols=bc)
    for H, R in zip(mats, ref):
        _same_factors(_factors(H), _factors(R))
        H.close()
        R.close()
