"""The black-box boundary of Alg. 1 through the C ABI: user sketch and entry
callbacks, h2_entries, the transposed h2_matvec, device export, the fixed
sample size of Sec. III-A and the Helmholtz volume-IE kernel (Sec. V-A).

Every case is compared with the oracle's construction of the same problem from
the same inputs (the oracle's own H^2 black boxes are built by the oracle):
identical sample counts, thresholds, ranks and skeletons; coupling and dense
blocks to entry rounding; the ID matrices to the rounding of the samples
amplified by the ID's conditioning (reported per depth).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_16759_amd as h2
from paper_2506_16759_amd.workloads import SMALL_2D, uniform_points
from oracle.build import build_h2
from oracle.kernels import CallbackOperator, KernelOperator
from gpu_util import (colmajor_from, compare_with_oracle, dense_from_matvec, fill_entry_batch, id_matrix_bar, say,
                      to_np)


@pytest.fixture(scope="module")
def ctx():
    return h2.Context(0)


def _oracle_old(pts, kind, length, leaf, tol, d0, seed):
    return build_h2(KernelOperator(pts, kind, length), pts, leaf, 0.7, tol, d0, 16, 256, seed)


def test_sketch_callback_h2_black_box(ctx):
    """Sec. V-A setting: the black box is the product with an existing H^2
    matrix, the blocks come from the kernel.  The GPU's H_old and the oracle's
    H_old are each built from the same recipe (and compared first)."""
    n, dim, leaf = 3000, 3, 48
    say(f"sketch callback = H2 matvec, n={n} dim={dim} leaf={leaf}")
    pts = uniform_points(n, dim, 501)
    H_old = h2.build(ctx, pts, "exp", 0.2, tol=1e-8, leaf_size=leaf, d0=32, d_inc=16, seed=7)
    ho_old = _oracle_old(pts, "exp", 0.2, leaf, 1e-8, 32, 7)
    compare_with_oracle(H_old, ho_old)
    calls = []

    def counted(om, y):
        calls.append(om.shape[1])
        y.copy_(H_old.matvec(om))

    H = h2.build(ctx, pts, "exp", 0.2, sketch=counted, tol=1e-6, leaf_size=leaf, d0=16, d_inc=16, seed=9,
                 sketch_ahead=0)
    info = H.info()
    op = CallbackOperator(n, ho_old.matvec, KernelOperator(pts, "exp", 0.2).entries)
    ho = build_h2(op, pts, leaf, 0.7, 1e-6, 16, 16, 256, 9)
    say(f"samples {info['samples']} (oracle {ho.samples}) rounds {info['rounds']} calls {calls}")
    assert info["samples"] == ho.samples
    assert abs(info["delta"] - ho.delta) <= 1e-12 * ho.delta
    assert info["sketch_calls"] == len(calls) == 1 + (ho.samples - 16) // 16
    assert sum(calls) == info["sketched"] == ho.samples
    diff = compare_with_oracle(H, ho)
    say(f"ID matrix differences per depth {diff}")
    x = np.random.default_rng(3).standard_normal((n, 3))
    y, yo = to_np(H.matvec(colmajor_from(x))), ho.matvec(x)
    assert np.linalg.norm(y - yo) / np.linalg.norm(yo) <= 1e-10
    assert info["sketch_flops"] == 0.0   # the library did not run its own sketch


def test_both_callbacks_exact_low_rank(ctx):
    """kernel = NULL: A = Phi Phi^T (rank 12) given only by its product and its
    entries, both on the device; recovered to rounding (exact low rank)."""
    import torch
    n, dim, r = 2500, 2, 12
    say(f"both callbacks, rank {r}, n={n}")
    pts = uniform_points(n, dim, 77)
    Phi = np.random.default_rng(5).standard_normal((n, r)) / np.sqrt(n)
    Pt = torch.from_numpy(Phi).cuda()
    seen = {"sketch": 0, "entry": 0}

    def sk(om, y):
        seen["sketch"] += 1
        y.copy_(Pt @ (Pt.T @ om))

    def en(batch):
        seen["entry"] += 1
        fill_entry_batch(batch, lambda i, j: (Pt[i] * Pt[j]).sum(dim=1))

    H = h2.build(ctx, pts, None, sketch=sk, entries=en, tol=1e-6, leaf_size=40, d0=16, d_inc=16, seed=21)
    info = H.info()
    op = CallbackOperator(n, lambda om: Phi @ (Phi.T @ om), lambda a, b: Phi[a] @ Phi[b].T)
    ho = build_h2(op, pts, 40, 0.7, 1e-6, 16, 16, 256, 21)
    say(f"samples {info['samples']} ranks {info['rank_min']}..{info['rank_max']} calls {seen}")
    assert info["samples"] == ho.samples
    assert info["rank_max"] <= r
    diff = compare_with_oracle(H, ho)
    # one entry call for the dense blocks and one per level with far blocks
    levels_with_far = sum(1 for t in range(ho.top, ho.tree.depth + 1) if len(ho.lists.far_idx[t]))
    assert seen["entry"] == 1 + levels_with_far
    A = Phi @ Phi.T
    KH = dense_from_matvec(H, n)
    err = np.linalg.norm(KH - A) / np.linalg.norm(A)
    say(f"reconstruction error {err:.3e}")
    assert err <= 1e-12


def test_h2_as_both_callbacks_and_entries(ctx):
    """Recompression of an H^2 matrix: the sketch is its product and the blocks
    its entries (h2_entries); the oracle does the same with its own H_old."""
    w = SMALL_2D
    say(f"H2 as sketch and entries, {w.name}")
    pts = w.points()
    H_old = h2.build(ctx, pts, w.kernel, w.length, tol=1e-8, leaf_size=w.leaf_size, d0=32, d_inc=16, seed=3)
    ho_old = _oracle_old(pts, w.kernel, w.length, w.leaf_size, 1e-8, 32, 3)
    compare_with_oracle(H_old, ho_old)
    # h2_entries against the oracle's entries of its own H_old, on rows and
    # columns that cross every kind of block
    rng = np.random.default_rng(4)
    rows, cols = rng.choice(w.n, 300, replace=False), rng.choice(w.n, 280, replace=False)
    eg = to_np(H_old.entries(rows, cols))
    eo = ho_old.entries(rows, cols)
    assert np.abs(eg - eo).max() <= 1e-12 * np.abs(eo).max()
    # and against the GPU's own product with unit vectors (same matrix)
    KH_old = dense_from_matvec(H_old, w.n)
    assert np.abs(eg - KH_old[np.ix_(rows, cols)]).max() <= 1e-13 * np.abs(eg).max()

    H = h2.build(ctx, pts, None, sketch=H_old, entries=H_old, tol=1e-6, leaf_size=w.leaf_size, d0=32, d_inc=16,
                 seed=w.omega_seed)
    info = H.info()
    ho = build_h2(CallbackOperator(w.n, ho_old.matvec, ho_old.entries), pts, w.leaf_size, w.eta, 1e-6, 32, 16,
                  256, w.omega_seed)
    assert info["samples"] == ho.samples
    # the coupling blocks are entries of the two sides' H_old, whose ID
    # matrices differ within their own bar
    diff = compare_with_oracle(H, ho, block_atol=id_matrix_bar(H_old))
    say(f"samples {info['samples']}, ID differences {diff}")
    KH = dense_from_matvec(H, w.n)
    err = np.linalg.norm(KH - KH_old) / np.linalg.norm(KH_old)
    say(f"recompression error {err:.3e}")
    assert err <= 10 * 1e-6


def test_entries_edge_cases(ctx):
    """h2_entries: single entries, repeated indices, a block with no rows, the
    diagonal, against the product with unit vectors."""
    import torch
    n = 1500
    say(f"h2_entries edge cases n={n}")
    pts = uniform_points(n, 3, 12)
    H = h2.build(ctx, pts, "gauss", 0.15, tol=1e-7, leaf_size=32, d0=32, d_inc=16, seed=1)
    KH = dense_from_matvec(H, n)
    for rows, cols in (([0], [0]), ([5, 5, 7], [9, 5]), (np.arange(n), [n - 1]), ([n - 1], np.arange(n))):
        e = to_np(H.entries(rows, cols))
        np.testing.assert_allclose(e, KH[np.ix_(rows, cols)], rtol=0, atol=1e-13 * np.abs(KH).max())
    assert H.entries([], [1, 2]).shape == (0, 2)
    # a batch of several blocks with ragged sizes through the raw call
    blocks = [(np.arange(10, 73), np.arange(100, 101)), (np.array([3]), np.arange(n)), (np.arange(0), np.arange(4)),
              (np.arange(700, 900), np.arange(1200, 1320))]
    idx, rb, rc, cb, cc, off = [], [], [], [], [], []
    pos = out_off = 0
    for r, c in blocks:
        rb.append(pos); rc.append(len(r)); idx.extend(r); pos += len(r)
        cb.append(pos); cc.append(len(c)); idx.extend(c); pos += len(c)
        off.append(out_off); out_off += len(r) * len(c)
    t = lambda v, dt: torch.tensor(v, dtype=dt, device="cuda")
    out = torch.full((out_off,), np.nan, dtype=torch.float64, device="cuda")
    args = [t(idx, torch.int32), t(rb, torch.int64), t(rc, torch.int32), t(cb, torch.int64), t(cc, torch.int32),
            t(off, torch.int64)]
    H.entries_raw(len(blocks), *(a.data_ptr() for a in args), out.data_ptr(), max(rc), max(cc))
    got = to_np(out)
    for (r, c), o in zip(blocks, off):
        ref = KH[np.ix_(r, c)]
        np.testing.assert_allclose(got[o:o + ref.size].reshape(len(c), len(r)).T, ref, rtol=0,
                                   atol=1e-13 * np.abs(KH).max())


def test_callback_failures_abort_cleanly(ctx):
    """A callback returning non-zero aborts the build with H2_ERR_CALLBACK, at
    the first sketch, in a later adaptive pass, or in the entry callback; the
    context stays usable."""
    import torch
    n = 2000
    pts = uniform_points(n, 3, 31)
    H_old = h2.build(ctx, pts, "exp", 0.2, tol=1e-8, leaf_size=32, seed=1)
    for fail_at in (1, 2):
        say(f"sketch callback fails at call {fail_at}")
        count = [0]

        def sk(om, y):
            count[0] += 1
            if count[0] == fail_at:
                raise RuntimeError("planted failure")
            y.copy_(H_old.matvec(om))

        with pytest.raises(h2.H2Error) as ei:
            h2.build(ctx, pts, "exp", 0.2, sketch=sk, tol=1e-8, leaf_size=32, d0=8, d_inc=8, sketch_ahead=0)
        assert ei.value.status == -4
        assert count[0] == fail_at
    for fail_at in (1, 2):
        say(f"entry callback fails at call {fail_at}")
        count = [0]

        def en(batch):
            count[0] += 1
            if count[0] == fail_at:
                raise RuntimeError("planted failure")
            H_old.entries_raw(batch.nblocks, *batch._ptrs, batch.max_rows, batch.max_cols)

        with pytest.raises(h2.H2Error) as ei:
            h2.build(ctx, pts, None, sketch=H_old, entries=en, tol=1e-6, leaf_size=32)
        assert ei.value.status == -4
    say("argument errors")
    with pytest.raises(h2.H2Error) as ei:      # entry callback without a sketch
        h2.build(ctx, pts, None, entries=H_old)
    assert ei.value.status == -1
    with pytest.raises(h2.H2Error) as ei:      # reduced precision needs the built-in sketch
        h2.build(ctx, pts, "exp", 0.2, sketch=H_old, precision=h2.BF16X6)
    assert ei.value.status == -7
    # the context still works
    H = h2.build(ctx, pts, "exp", 0.2, tol=1e-6, leaf_size=32)
    K = KernelOperator(pts, "exp", 0.2)
    x = np.random.default_rng(2).standard_normal(n)
    y = to_np(H.matvec(torch.from_numpy(x).cuda()))
    assert np.linalg.norm(y - K.sketch(x[:, None])[:, 0]) <= 1e-5 * np.linalg.norm(y)


def test_matvec_transpose_and_device_export(ctx):
    """trans = 1 of a symmetric build is the same product; exported parts are
    the same on the host and on the device."""
    import torch
    n = 3500
    say(f"transpose and device export n={n}")
    pts = uniform_points(n, 3, 8)
    H = h2.build(ctx, pts, "exp", 0.2, tol=1e-6, leaf_size=48, seed=4)
    x = colmajor_from(np.random.default_rng(6).standard_normal((n, 5)))
    np.testing.assert_array_equal(to_np(H.matvec(x, trans=True)), to_np(H.matvec(x)))
    D, top = int(H.export("DEPTH")[0]), int(H.export("TOP")[0])
    for name in ("PERM", "NODES", "BOXES", "NEAR_PTR", "NEAR_IDX", "DENSE", "TOP", "DEPTH"):
        np.testing.assert_array_equal(to_np(H.export(name, device=True)), H.export(name))
    for t in range(top, D + 1):
        for name in ("FAR_PTR", "FAR_IDX", "RANKS", "SKEL", "SKEL_POS", "BASIS", "COUPLING"):
            np.testing.assert_array_equal(to_np(H.export(name, t, device=True)), H.export(name, t))


def test_fixed_sample_size_matches_oracle(ctx):
    """Sec. III-A: exactly d0 columns, no convergence test, no adaptive rounds."""
    w = SMALL_2D
    for d0 in (24, 64):
        say(f"fixed sample size d0={d0}, {w.name}")
        pts = w.points()
        H = h2.build(ctx, pts, w.kernel, w.length, tol=w.tol, leaf_size=w.leaf_size, eta=w.eta, d0=d0, d_inc=0,
                     seed=w.omega_seed)
        info = H.info()
        assert info["samples"] == d0 and info["rounds"] == 0 and info["fixed_samples"] == 1
        assert info["sketch_calls"] == 1 and info["sketched"] == d0
        op = KernelOperator(pts, w.kernel, w.length)
        ho = build_h2(op, pts, w.leaf_size, w.eta, w.tol, d0, 0, 256, w.omega_seed)
        assert ho.samples == d0
        diff = compare_with_oracle(H, ho)
        say(f"ranks {info['rank_min']}..{info['rank_max']}, ID differences {diff}")
        K = op.dense()
        eF = np.linalg.norm(K - dense_from_matvec(H, w.n)) / np.linalg.norm(K)
        eo = np.linalg.norm(K - ho.dense()) / np.linalg.norm(K)
        say(f"eF={eF:.3e} (oracle {eo:.3e})")
        assert abs(eF - eo) <= 1e-3 * eo + 1e-14


# ------------------------------------------------------------------ Helmholtz IE kernel
@pytest.mark.parametrize("n,dim,k,ncols", [(1000, 3, 3.0, 32), (2049, 3, 3.0, 17), (333, 2, 10.0, 5)])
def test_helmholtz_sketch_and_blocks(ctx, n, dim, k, ncols):
    import torch
    say(f"helmholtz sketch n={n} dim={dim} k={k} ncols={ncols}")
    pts = uniform_points(n, dim, 900 + n)
    pts[:, 7] = pts[:, 3]                 # a coincident pair: its entries are 0 like the diagonal
    om = np.random.default_rng(n).standard_normal((n, ncols))
    y = to_np(h2.sketch(ctx, torch.from_numpy(pts), "helmholtz", k, colmajor_from(om)))
    op = KernelOperator(pts, "helmholtz", k)
    ref = op.sketch(om)
    scale = np.abs(ref).max(axis=0)
    rel = (np.abs(y - ref).max(axis=0) / scale).max()
    say(f"column-relative sketch error {rel:.3e}")
    assert rel <= 1e-12
    with pytest.raises(h2.H2Error) as ei:
        h2.sketch(ctx, torch.from_numpy(pts), "helmholtz", k, colmajor_from(om), precision=h2.FP32)
    assert ei.value.status == -7


def test_helmholtz_build_matches_oracle(ctx):
    """cos(3r)/r on 3D points (Table II's IE problem at a small size): tree and
    lists, ranks, skeletons and blocks as the oracle's, accuracy against the
    dense operator."""
    n, dim, kw, leaf, tol = 4096, 3, 3.0, 64, 1e-6
    say(f"helmholtz build n={n} k={kw} tol={tol}")
    pts = uniform_points(n, dim, 1234)
    H = h2.build(ctx, pts, "helmholtz", wavenumber=kw, tol=tol, leaf_size=leaf, d0=32, d_inc=16, seed=1003)
    info = H.info()
    op = KernelOperator(pts, "helmholtz", kw)
    ho = build_h2(op, pts, leaf, 0.7, tol, 32, 16, 256, 1003)
    assert info["samples"] == ho.samples
    diff = compare_with_oracle(H, ho)
    K = op.dense()
    KH = dense_from_matvec(H, n)
    eF = np.linalg.norm(K - KH) / np.linalg.norm(K)
    say(f"samples {info['samples']} ranks {info['rank_min']}..{info['rank_max']} eF={eF:.3e} ID diff {diff}")
    assert eF <= 10 * tol
    assert np.linalg.norm(KH - ho.dense()) / np.linalg.norm(K) <= 1e-10
