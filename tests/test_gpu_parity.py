"""GPU parity of the HIP construction path against the FP64 oracle.

Every case prints its name, sizes and seeds before touching the GPU.  Floating
point tolerances:
  * Omega: both sides evaluate the same Philox words; only log/cos/sqrt of the
    two math libraries differ (a few ulps)  ->  |diff| <= 1e-13.
  * dense sketch: same products summed in a different order, kernel entries
    within a few ulps  ->  relative (to the column's max) <= 1e-12.
  * dense blocks D: same formula, exp/sqrt ulps  ->  relative <= 1e-13.
  * whole construction against the exact K: the accuracy bound (relative
    Frobenius and matvec error <= 10 tol), plus structural identities
    (tree/lists bit-exact, U(J,:) = I exactly);
  * whole construction against the oracle's construction of the same problem
    with the same Omega: identical sample count, rounds, threshold, ranks and
    skeletons; coupling and dense blocks to entry rounding (1e-12 / 1e-13);
    ID matrices U = P^T [I; T^T] within 1e-9 of each node's largest entry (the
    samples differ by summation-order rounding, which the triangular solve for
    T amplifies by cond(R11) <~ ||Y|| / delta); products within 1e-10.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_16759_amd as h2
from paper_2506_16759_amd.workloads import CUBE_131K, SMALL_2D, gaussian_vectors, uniform_points
from oracle.build import build_h2
from oracle.kernels import KernelOperator
from oracle.philox import gaussian as oracle_gaussian
from oracle.tree import build_lists, build_tree
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


def _dense_from_matvec(H, n):
    import torch
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    return _np(H.matvec(eye.T.contiguous().T))


@pytest.mark.parametrize("n,col0,ncols,seed", [(1, 0, 1, 1), (1000, 0, 32, 1000), (4099, 48, 17, 7),
                                               (70000, 5, 3, 123456789)])
def test_gaussian_matches_oracle(ctx, n, col0, ncols, seed):
    import torch
    _say(f"gaussian n={n} col0={col0} ncols={ncols} seed={seed}")
    rows = np.random.default_rng(n).permutation(max(n, 1) * 3)[:n].astype(np.int32)
    out = _np(h2.gaussian(ctx, seed, torch.from_numpy(rows), col0, ncols))
    ref = oracle_gaussian(seed, rows, col0, ncols)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n,dim,kind,length,ncols", [
    (1000, 2, "exp", 0.1, 32), (3001, 3, "exp", 0.2, 48), (777, 3, "gauss", 0.15, 16), (129, 1, "exp", 0.3, 1),
    (2500, 2, "gauss", 0.05, 80), (4096, 3, "exp", 0.2, 64), (200, 3, "exp", 0.2, 20),
])
def test_sketch_matches_oracle(ctx, n, dim, kind, length, ncols):
    _say(f"sketch n={n} dim={dim} kernel={kind} l={length} ncols={ncols}")
    pts = uniform_points(n, dim, 10 + n)
    om = np.random.default_rng(n).standard_normal((n, ncols))
    import torch
    y = _np(h2.sketch(ctx, torch.from_numpy(pts), kind, length, _colmajor_from(om)))
    ref = KernelOperator(pts, kind, length).sketch(om)
    scale = np.abs(ref).max(axis=0)
    assert (np.abs(y - ref).max(axis=0) <= 1e-12 * scale).all()


def _check_tree_lists(H, pts, leaf, eta):
    tr = build_tree(pts, leaf)
    L = build_lists(tr, eta)
    D = int(H.export("DEPTH")[0])
    assert D == tr.depth
    np.testing.assert_array_equal(H.export("PERM"), tr.perm)
    np.testing.assert_array_equal(H.export("NEAR_PTR"), L.near_ptr)
    np.testing.assert_array_equal(H.export("NEAR_IDX"), L.near_idx)
    for t in range(D + 1):
        np.testing.assert_array_equal(H.export("FAR_PTR", t), L.far_ptr[t])
        np.testing.assert_array_equal(H.export("FAR_IDX", t), L.far_idx[t])
    return tr, L


def _check_identity_rows(H):
    """U(J,:) = I exactly at every processed depth (the ID invariant)."""
    D = int(H.export("DEPTH")[0])
    top = int(H.export("TOP")[0])
    nodes = H.export("NODES").reshape(-1, 2)
    for t in range(top, D + 1):
        ranks = H.export("RANKS", t)
        basis = H.export("BASIS", t)
        skel = H.export("SKEL_POS", t)
        if t == D:
            m = np.array([nodes[(1 << D) - 1 + i, 1] - nodes[(1 << D) - 1 + i, 0] for i in range(1 << D)])
            rows_of = [np.arange(nodes[(1 << D) - 1 + i, 0], nodes[(1 << D) - 1 + i, 1]) for i in range(1 << D)]
        else:
            kc = H.export("RANKS", t + 1)
            sk_c = H.export("SKEL_POS", t + 1)
            offc = np.concatenate([[0], np.cumsum(kc)])
            m = kc[0::2] + kc[1::2]
            rows_of = [sk_c[offc[2 * i]:offc[2 * i + 2]] for i in range(1 << t)]
        off_b, off_s = 0, 0
        for i in range(1 << t):
            k = int(ranks[i])
            U = basis[off_b:off_b + m[i] * k].reshape(k, m[i]).T
            sk = skel[off_s:off_s + k]
            J = np.array([np.nonzero(rows_of[i] == s)[0][0] for s in sk], dtype=int)
            np.testing.assert_array_equal(U[J], np.eye(k))
            off_b += m[i] * k
            off_s += k
        assert off_b == basis.size and off_s == skel.size


def test_build_small_2d_parity(ctx):
    w = SMALL_2D
    _say(f"build {w.name} n={w.n} tol={w.tol}")
    pts = w.points()
    H = h2.build(ctx, pts, w.kernel, w.length, tol=w.tol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0,
                 d_inc=w.d_inc, seed=w.omega_seed)
    info = H.info()
    _check_tree_lists(H, pts, w.leaf_size, w.eta)
    _check_identity_rows(H)
    op = KernelOperator(pts, w.kernel, w.length)
    K = op.dense()
    KH = _dense_from_matvec(H, w.n)
    eF = np.linalg.norm(K - KH) / np.linalg.norm(K)
    x = np.random.default_rng(8).standard_normal((w.n, 8))
    y = _np(H.matvec(_colmajor_from(x)))
    emv = np.linalg.norm(K @ x - y) / np.linalg.norm(K @ x)
    _say(f"eF={eF:.3e} emv={emv:.3e} samples={info['samples']} ranks={info['rank_min']}..{info['rank_max']}")
    assert eF <= 10 * w.tol and emv <= 10 * w.tol
    # against the oracle's own construction of the same problem with the same
    # Omega: same samples, threshold, ranks and skeletons; blocks to entry
    # rounding; ID matrices to the samples' rounding times the ID conditioning
    ho = build_h2(op, pts, w.leaf_size, w.eta, w.tol, w.d0, w.d_inc, 128, w.omega_seed)
    assert info["samples"] == ho.samples
    assert abs(info["delta"] - ho.delta) <= 1e-12 * ho.delta
    diff = compare_with_oracle(H, ho)
    _say(f"ID matrix differences per depth {diff}")
    eo = np.linalg.norm(KH - ho.dense()) / np.linalg.norm(K)
    _say(f"||K_H - K_H(oracle)|| / ||K|| = {eo:.3e}")
    assert eo <= 1e-10


@pytest.mark.parametrize("n,dim,kind,length,leaf,tol,d0,seed", [
    (6000, 3, "exp", 0.2, 64, 1e-7, 16, 11),     # two adaptive rounds at the leaves
    (16384, 3, "exp", 0.2, 64, 1e-6, 32, 11),    # 3D, 256 leaves, one round
    (5000, 2, "gauss", 0.1, 50, 1e-6, 16, 12),   # ragged leaves, Gaussian kernel
])
def test_build_matches_oracle_with_rounds(ctx, n, dim, kind, length, leaf, tol, d0, seed):
    """The adaptive loop (updateSamples: draw, sweep up through the finished
    levels, test again) against the oracle's construction of the same problem,
    factor by factor."""
    _say(f"oracle parity with rounds n={n} dim={dim} {kind} l={length} leaf={leaf} tol={tol} d0={d0}")
    pts = uniform_points(n, dim, 40 + n)
    H = h2.build(ctx, pts, kind, length, tol=tol, leaf_size=leaf, eta=0.7, d0=d0, d_inc=16, seed=seed)
    info = H.info()
    op = KernelOperator(pts, kind, length)
    ho = build_h2(op, pts, leaf, 0.7, tol, d0, 16, 256, seed)
    _say(f"samples {info['samples']} (oracle {ho.samples}), rounds {info['rounds']} (oracle {ho.rounds}), "
         f"ranks {info['rank_min']}..{info['rank_max']}")
    _check_tree_lists(H, pts, leaf, 0.7)
    assert info["samples"] == ho.samples
    assert info["rounds"] == sum(ho.rounds.values())
    assert abs(info["delta"] - ho.delta) <= 1e-12 * ho.delta
    diff = compare_with_oracle(H, ho)
    _say(f"ID matrix differences per depth {diff}")
    x = np.random.default_rng(2).standard_normal((n, 4))
    y, yo = _np(H.matvec(_colmajor_from(x))), ho.matvec(x)
    emv = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    kx = op.sketch(x)
    e_exact = np.linalg.norm(y - kx) / np.linalg.norm(kx)
    _say(f"matvec vs oracle {emv:.3e}, vs exact {e_exact:.3e}")
    assert emv <= 1e-10
    assert e_exact <= 10 * tol


@pytest.mark.parametrize("n,dim,kind,length,leaf,tol,d0,dinc", [
    (6000, 3, "exp", 0.2, 64, 1e-7, 16, 16),     # forces adaptive rounds
    (3333, 2, "gauss", 0.1, 40, 1e-6, 32, 16),   # ragged leaves, Gaussian kernel
    (2048, 3, "exp", 0.2, 32, 1e-8, 32, 16),
])
def test_build_matches_dense_bound(ctx, n, dim, kind, length, leaf, tol, d0, dinc):
    _say(f"build n={n} dim={dim} {kind} l={length} leaf={leaf} tol={tol} d0={d0}+{dinc}")
    pts = uniform_points(n, dim, 40 + n)
    H = h2.build(ctx, pts, kind, length, tol=tol, leaf_size=leaf, eta=0.7, d0=d0, d_inc=dinc, seed=11)
    info = H.info()
    _check_tree_lists(H, pts, leaf, 0.7)
    _check_identity_rows(H)
    K = KernelOperator(pts, kind, length).dense()
    KH = _dense_from_matvec(H, n)
    eF = np.linalg.norm(K - KH) / np.linalg.norm(K)
    _say(f"eF={eF:.3e} samples={info['samples']} rounds={info['rounds']} ranks={info['rank_min']}..{info['rank_max']}")
    assert eF <= 10 * tol


@pytest.mark.parametrize("n,leaf", [(1440, 96), (1100, 150), (3000, 64)])
def test_dense_blocks_are_kernel_entries(ctx, n, leaf):
    """Every near-field block equals the kernel on its clusters' points, for
    leaf heights the block generator lays out as fixed rows per thread (64)
    and as entries in order (90 and 137/138 rows)."""
    pts = uniform_points(n, 3, 70 + leaf)
    _say(f"dense blocks: n={n} leaf={leaf}")
    H = h2.build(ctx, pts, "exp", 0.2, tol=1e-6, leaf_size=leaf, eta=0.7, d0=16, d_inc=16, seed=3)
    D = int(H.export("DEPTH")[0])
    nodes = H.export("NODES").reshape(-1, 2)
    perm = H.export("PERM")
    npp, ni = H.export("NEAR_PTR"), H.export("NEAR_IDX")
    Dg = H.export("DENSE")
    x = np.asarray(pts)[:, perm]   # tree order
    heights = set()
    off = 0
    for s in range(1 << D):
        bs, es = nodes[(1 << D) - 1 + s]
        heights.add(int(es - bs))
        for j in range(npp[s], npp[s + 1]):
            b = int(ni[j])
            bb, eb = nodes[(1 << D) - 1 + b]
            d2 = ((x[:, bs:es, None] - x[:, None, bb:eb]) ** 2).sum(axis=0)
            ref = np.exp(-np.sqrt(d2) / 0.2)
            got = Dg[off:off + ref.size].reshape(eb - bb, es - bs).T
            np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-300)
            off += ref.size
    assert off == Dg.size
    # the near-field products of the build and of the matvec run on these
    # block heights too (rows beyond 64 in 64-row slices)
    K = KernelOperator(pts, "exp", 0.2).dense()
    eF = np.linalg.norm(K - _dense_from_matvec(H, n)) / np.linalg.norm(K)
    _say(f"leaf heights {sorted(heights)}, eF={eF:.3e}")
    assert eF <= 10 * 1e-6
    H.close()


def test_edge_cases(ctx):
    import torch
    _say("edge: single leaf, nothing admissible, duplicates, n=1")
    pts = uniform_points(50, 2, 1)
    H = h2.build(ctx, pts, "exp", 0.2, leaf_size=64)
    K = KernelOperator(pts, "exp", 0.2).dense()
    np.testing.assert_allclose(_dense_from_matvec(H, 50), K, rtol=1e-14, atol=1e-15)
    pts = uniform_points(600, 2, 2)
    H = h2.build(ctx, pts, "gauss", 0.2, leaf_size=16, eta=1e-9)
    assert H.info()["samples"] == 0
    np.testing.assert_allclose(_dense_from_matvec(H, 600), KernelOperator(pts, "gauss", 0.2).dense(),
                               rtol=1e-13, atol=1e-15)
    pts = np.repeat(uniform_points(700, 3, 3), 2, axis=1)
    H = h2.build(ctx, pts, "exp", 0.2, leaf_size=32, tol=1e-6)
    K = KernelOperator(pts, "exp", 0.2).dense()
    assert np.linalg.norm(K - _dense_from_matvec(H, 1400)) / np.linalg.norm(K) <= 1e-5
    H = h2.build(ctx, np.array([[0.5], [0.25]]), "exp", 0.2)
    assert abs(_np(H.matvec(torch.ones(1, dtype=torch.float64, device="cuda")))[0] - 1.0) < 1e-15


def test_sample_limit_is_reported(ctx):
    _say("error path: d_max reached")
    pts = uniform_points(3000, 3, 6)
    with pytest.raises(h2.H2Error) as ei:
        h2.build(ctx, pts, "exp", 0.2, leaf_size=48, tol=1e-10, d0=8, d_inc=8, d_max=16)
    assert ei.value.status == -5


def test_full_size_cube_sampled_parity(ctx):
    """The timed workload at full size: bit-exact tree/lists, sampled sketch rows,
    sampled matvec rows against the oracle's dense products."""
    import torch
    w = CUBE_131K
    _say(f"full size {w.name} n={w.n} tol={w.tol}")
    pts = w.points()
    H = h2.build(ctx, pts, w.kernel, w.length, tol=w.tol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0,
                 d_inc=w.d_inc, seed=w.omega_seed)
    info = H.info()
    _say(f"built: {info['t_total']:.1f} ms samples={info['samples']} ranks={info['rank_min']}..{info['rank_max']}")
    _check_tree_lists(H, pts, w.leaf_size, w.eta)
    op = KernelOperator(pts, w.kernel, w.length)
    rng = np.random.default_rng(17)
    rows = rng.choice(w.n, 64, replace=False)
    # sketch at full size, sampled rows
    om = np.random.default_rng(5).standard_normal((w.n, 32))
    y = _np(h2.sketch(ctx, torch.from_numpy(pts), w.kernel, w.length, _colmajor_from(om)))
    ref = op.sketch_rows(rows, om)
    assert np.abs(y[rows] - ref).max() <= 1e-12 * np.abs(ref).max()
    # H^2 matvec against the exact dense product on sampled rows
    x = np.random.default_rng(9).standard_normal((w.n, 4))
    yh = _np(H.matvec(_colmajor_from(x)))
    kx = op.entries(rows, np.arange(w.n)) @ x
    emv = np.linalg.norm(yh[rows] - kx) / np.linalg.norm(kx)
    _say(f"sampled-row matvec error {emv:.3e}")
    assert emv <= 10 * w.tol


CUBE_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube_exp3d_n131072_tol{:.0e}.json")


@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_full_size_cube_matches_oracle_golden(ctx, tol):
    """The benchmarked 131072-point cube at tol 1e-6 and 1e-8 against the
    oracle's construction of it (stored by tests/golden/make_cube_golden.py,
    which runs only the oracle): the same sample count, threshold, top depth
    and ranks of all 4094 clusters, the same skeleton index sets at every
    depth (SHA-256 of the SKEL export), and sampled products within 1e-10 of
    the oracle's H^2 matrix and within 10 tol of the exact kernel."""
    import hashlib
    path = CUBE_GOLDEN.format(tol)
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} not written yet (tests/golden/make_cube_golden.py)")
    g = json.load(open(path))
    w = CUBE_131K
    _say(f"full size {w.name} tol={tol} against the stored oracle construction")
    pts = w.points()
    H = h2.build(ctx, pts, w.kernel, w.length, tol=tol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0, d_inc=w.d_inc,
                 d_max=g["d_max"], seed=w.omega_seed)
    info = H.info()
    _say(f"built: {info['t_total']:.1f} ms samples={info['samples']} (oracle {g['samples']}) "
         f"ranks={info['rank_min']}..{info['rank_max']}")
    assert info["samples"] == g["samples"]
    assert abs(info["delta"] - g["delta"]) <= 1e-12 * g["delta"]
    assert int(H.export("TOP")[0]) == g["top"]
    for t, ko in g["ranks"].items():
        np.testing.assert_array_equal(H.export("RANKS", int(t)), np.array(ko), err_msg=f"ranks at depth {t}")
    for t, sha in g["skel_sha256"].items():
        got = hashlib.sha256(H.export("SKEL", int(t)).astype("<i4").tobytes()).hexdigest()
        assert got == sha, f"skeletons at depth {t}"
    rows = np.array(g["rows"])
    x = gaussian_vectors(w.n, 4, g["x_seed"])
    y = _np(H.matvec(_colmajor_from(x)))[rows]
    y_or, y_ex = np.array(g["y_h2"]), np.array(g["y_exact"])
    e_or = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
    e_ex = np.linalg.norm(y - y_ex) / np.linalg.norm(y_ex)
    _say(f"sampled rows: vs oracle H^2 {e_or:.3e}, vs exact kernel {e_ex:.3e}")
    assert e_or <= 1e-10
    assert e_ex <= 10 * tol
    H.close()


# ------------------------------------------------------------------ mixed precision
# FP32 entries carry ~1e-7 relative error; FP32 partial sums are folded into
# FP64 every 64 points (precisions 1, 2, 4), so each sketch column stays within
# a few 1e-7 of its max; bf16x3 products carry ~2^-17 relative error, bf16x6
# products ~2^-24; FP32 entries contracted in FP64 (precision 3) leave only the
# entry noise.  The bars below leave a factor of ~10 over those estimates.
MIXED_TOL = {1: 1e-5, 2: 2e-3, 3: 1e-6, 4: 1e-5}


@pytest.mark.parametrize("precision", [1, 2, 3, 4])
@pytest.mark.parametrize("n,dim,kind,length,ncols", [
    (1000, 2, "exp", 0.1, 32), (3001, 3, "exp", 0.2, 48), (777, 3, "gauss", 0.15, 16), (129, 1, "exp", 0.3, 1),
    (2500, 2, "gauss", 0.05, 80), (4096, 3, "exp", 0.2, 64),
])
def test_sketch_mixed_precision(ctx, precision, n, dim, kind, length, ncols):
    import torch
    _say(f"sketch precision={precision} n={n} dim={dim} kernel={kind} l={length} ncols={ncols}")
    pts = uniform_points(n, dim, 10 + n)
    om = np.random.default_rng(n).standard_normal((n, ncols))
    y = _np(h2.sketch(ctx, torch.from_numpy(pts), kind, length, _colmajor_from(om), precision=precision))
    ref = KernelOperator(pts, kind, length).sketch(om)
    rel = (np.abs(y - ref).max(axis=0) / np.abs(ref).max(axis=0)).max()
    _say(f"max column-relative error {rel:.3e}")
    assert rel <= MIXED_TOL[precision]


@pytest.mark.parametrize("precision,tol", [(1, 1e-6), (2, 1e-4), (1, 1e-4), (3, 1e-6), (3, 1e-8), (4, 1e-6), (4, 1e-4)])
def test_build_mixed_precision_meets_tol(ctx, precision, tol):
    n, dim, kind, length = 6000, 3, "exp", 0.2
    _say(f"build precision={precision} tol={tol} n={n}")
    pts = uniform_points(n, dim, 77)
    H = h2.build(ctx, pts, kind, length, tol=tol, leaf_size=64, eta=0.7, d0=32, d_inc=16, seed=5,
                 precision=precision)
    info = H.info()
    _check_tree_lists(H, pts, 64, 0.7)
    _check_identity_rows(H)
    K = KernelOperator(pts, kind, length).dense()
    KH = _dense_from_matvec(H, n)
    eF = np.linalg.norm(K - KH) / np.linalg.norm(K)
    _say(f"eF={eF:.3e} samples={info['samples']} ranks={info['rank_min']}..{info['rank_max']}")
    assert eF <= 10 * tol


@pytest.mark.parametrize("precision,tol", [(4, 1e-6), (1, 1e-6), (2, 1e-4)])
def test_full_size_cube_mixed_precision_sampled(ctx, precision, tol):
    """The timed workload at full size in the reduced-precision modes that the
    benchmark times: every sketch in BF16X6 / FP32 at 1e-6 and bf16x3 at 1e-4,
    checked on sampled rows of the matvec against the exact kernel rows, and
    the sample count of the FP64 build at the same tolerance."""
    w = CUBE_131K
    pts = w.points()
    _say(f"full size {w.name} precision={precision} tol={tol}")
    H = h2.build(ctx, pts, w.kernel, w.length, tol=tol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0,
                 d_inc=w.d_inc, seed=w.omega_seed, precision=precision)
    info = H.info()
    _say(f"built: {info['t_total']:.1f} ms samples={info['samples']} ranks={info['rank_min']}..{info['rank_max']}")
    _check_tree_lists(H, pts, w.leaf_size, w.eta)
    H64 = h2.build(ctx, pts, w.kernel, w.length, tol=tol, leaf_size=w.leaf_size, eta=w.eta, d0=w.d0,
                   d_inc=w.d_inc, seed=w.omega_seed)
    assert info["samples"] == H64.info()["samples"]
    op = KernelOperator(pts, w.kernel, w.length)
    rows = np.random.default_rng(23).choice(w.n, 48, replace=False)
    x = np.random.default_rng(29).standard_normal((w.n, 3))
    kx = op.entries(rows, np.arange(w.n)) @ x
    e = np.linalg.norm(_np(H.matvec(_colmajor_from(x)))[rows] - kx) / np.linalg.norm(kx)
    e64 = np.linalg.norm(_np(H64.matvec(_colmajor_from(x)))[rows] - kx) / np.linalg.norm(kx)
    _say(f"sampled-row matvec error {e:.3e} (FP64 build {e64:.3e})")
    assert e <= 10 * tol
    H.close()
    H64.close()


def test_sketch_ahead_does_not_change_the_result(ctx):
    """Columns sketched ahead of need are used exactly as if drawn lazily: the
    construction is identical for any look-ahead (Omega is counter-based)."""
    n = 6000
    _say(f"sketch-ahead invariance n={n}")
    pts = uniform_points(n, 3, 91)
    outs = []
    for ahead in (0, 16, 64):
        H = h2.build(ctx, pts, "exp", 0.2, tol=1e-7, leaf_size=64, eta=0.7, d0=16, d_inc=16, seed=3,
                     sketch_ahead=ahead)
        info = H.info()
        D, top = int(H.export("DEPTH")[0]), int(H.export("TOP")[0])
        outs.append((info["samples"], info["rounds"],
                     [H.export("RANKS", t) for t in range(top, D + 1)],
                     [H.export("SKEL", t) for t in range(top, D + 1)],
                     [H.export("BASIS", t) for t in range(top, D + 1)],
                     [H.export("COUPLING", t) for t in range(top, D + 1)]))
        _say(f"ahead={ahead}: samples={info['samples']} sketched={info['sketched']} rounds={info['rounds']}")
    base = outs[0]
    for o in outs[1:]:
        assert o[0] == base[0] and o[1] == base[1]
        for a, b in zip(o[2], base[2]):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(o[3], base[3]):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(o[4] + o[5], base[4] + base[5]):
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("precision", ["FP64", "BF16X6", "FP64_SYM"])
def test_repeated_builds_are_bit_identical(ctx, precision):
    """Two builds of the same problem give the same matrix bit for bit (no
    atomics or scheduling-dependent sums on the path), so the benchmark may
    measure accuracy on a build after its timed ones."""
    n = 20000
    _say(f"repeated builds n={n} precision={precision}")
    pts = uniform_points(n, 3, 92)
    outs = []
    for _ in range(2):
        H = h2.build(ctx, pts, "exp", 0.2, tol=1e-6, leaf_size=64, eta=0.7, d0=32, d_inc=16, seed=4,
                     precision=getattr(h2, precision))
        D, top = int(H.export("DEPTH")[0]), int(H.export("TOP")[0])
        outs.append([H.export(part, t) for t in range(top, D + 1) for part in ("RANKS", "SKEL", "BASIS", "COUPLING")]
                    + [H.export("DENSE")])
        H.close()
    assert len(outs[0]) == len(outs[1])
    for a, b in zip(outs[0], outs[1]):
        assert a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))
