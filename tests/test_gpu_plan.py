"""Device planner (h2_plan_create_device) against the host planner.

The host planner's tree and lists equal the oracle's bit for bit
(tests/test_lib_host.py); the device planner must give the same plan bit for
bit: permutation, node ranges, boxes (compared as bit patterns), near lists
and far lists at every depth.  Cases cover 1-3 dimensions, ragged sizes, a
single leaf, the smallest leaf size and the largest, several eta, lattice
points with many equal coordinates (ties broken by original index), duplicate
points, signed zeros, clustered and wide-range clouds, and the
131072-point cube.
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_16759_amd as h2
from paper_2506_16759_amd.workloads import uniform_points


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return h2.Context(0)


def _lattice(n, dim, k, seed):
    """n points on a k^dim lattice (many equal coordinates and duplicates)."""
    g = np.random.default_rng(seed).integers(0, k, size=(dim, n))
    return g.astype(np.float64) / k


def _clusters(n, dim, seed):
    rng = np.random.default_rng(seed)
    centres = rng.random((8, dim))
    lab = rng.integers(0, 8, n)
    return (centres[lab] + 1e-3 * rng.standard_normal((n, dim))).T.copy()


def _signed_zeros(n, dim, seed):
    x = np.random.default_rng(seed).integers(-2, 3, size=(dim, n)).astype(np.float64) * 0.5
    x[x == 0] = np.where(np.random.default_rng(seed + 1).random(np.count_nonzero(x == 0)) < 0.5, -0.0, 0.0)
    return x


def _wide(n, dim, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((dim, n)) * 10.0 ** rng.integers(-6, 7, size=(dim, n))).astype(np.float64)


CASES = [
    # (label, points generator, leaf, eta)
    ("uniform 3d 5000", lambda: uniform_points(5000, 3, 1), 64, 0.7),
    ("uniform 2d 4096", lambda: uniform_points(4096, 2, 0), 64, 0.7),
    ("uniform 1d 3001", lambda: uniform_points(3001, 1, 2), 32, 0.7),
    ("uniform 3d 777 leaf 24", lambda: uniform_points(777, 3, 3), 24, 0.5),
    ("uniform 2d 2 leaf 2", lambda: uniform_points(2, 2, 4), 2, 0.7),
    ("single leaf", lambda: uniform_points(50, 3, 5), 64, 0.7),
    ("leaf 2", lambda: uniform_points(1000, 2, 6), 2, 0.7),
    ("leaf 256", lambda: uniform_points(70000, 3, 7), 256, 0.7),
    ("eta 2", lambda: uniform_points(6000, 3, 8), 48, 2.0),
    ("eta 0.3", lambda: uniform_points(6000, 2, 9), 40, 0.3),
    ("lattice 3d", lambda: _lattice(20000, 3, 9, 10), 64, 0.7),
    ("lattice 2d coarse", lambda: _lattice(5000, 2, 3, 11), 16, 0.7),
    ("lattice 1d", lambda: _lattice(4000, 1, 50, 12), 32, 0.7),
    ("duplicates", lambda: np.repeat(uniform_points(300, 3, 13), 7, axis=1), 32, 0.7),
    ("signed zeros", lambda: _signed_zeros(3000, 3, 14), 32, 0.7),
    ("clusters", lambda: _clusters(10000, 3, 15), 64, 0.7),
    ("wide range", lambda: _wide(8000, 2, 16), 64, 0.7),
]


def _compare(ph, pd):
    D = int(ph.export("DEPTH")[0])
    assert int(pd.export("DEPTH")[0]) == D
    for part in ("PERM", "NODES", "NEAR_PTR", "NEAR_IDX"):
        a, b = ph.export(part), pd.export(part)
        assert a.dtype == b.dtype and np.array_equal(a, b), part
    bh, bd = ph.export("BOXES"), pd.export("BOXES")
    assert np.array_equal(bh.view(np.uint64), bd.view(np.uint64)), "BOXES"
    for t in range(D + 1):
        for part in ("FAR_PTR", "FAR_IDX"):
            assert np.array_equal(ph.export(part, t), pd.export(part, t)), (part, t)
    return D


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_device_plan_equals_host_plan(ctx, case):
    label, gen, leaf, eta = case
    pts = gen()
    _say(f"device plan {label}: n={pts.shape[1]} dim={pts.shape[0]} leaf={leaf} eta={eta}")
    ph = h2.plan_create(pts, leaf, eta)
    pd = h2.plan_create(pts, leaf, eta, ctx=ctx)
    D = _compare(ph, pd)
    _say(f"  depth {D}, near blocks {len(ph.export('NEAR_IDX'))}: equal")


def test_device_plan_full_size_cube(ctx):
    """The 131072-point cube (leaf 64, eta 0.7) and its timing against the host planner."""
    import torch
    pts = uniform_points(131072, 3, 1)
    dp = torch.from_numpy(pts).cuda()
    _say("device plan 131072-point cube")
    h2.plan_create(dp, 64, 0.7, ctx=ctx)  # warm-up (code objects, pools)
    t0 = time.perf_counter()
    pd = h2.plan_create(dp, 64, 0.7, ctx=ctx)
    t_dev = time.perf_counter() - t0
    t0 = time.perf_counter()
    ph = h2.plan_create(pts, 64, 0.7)
    t_host = time.perf_counter() - t0
    _compare(ph, pd)
    _say(f"  equal; device {t_dev * 1e3:.2f} ms, host {t_host * 1e3:.2f} ms")


def test_device_plan_rejects_bad_input(ctx):
    pts = uniform_points(1000, 3, 1)
    pts[1, 17] = np.nan
    with pytest.raises(h2.H2Error) as e:
        h2.plan_create(pts, 64, 0.7, ctx=ctx)
    assert e.value.status == -1 and "finite" in str(e.value)
    with pytest.raises(h2.H2Error) as e:
        h2.plan_create(uniform_points(100, 3, 1), 1, 0.7, ctx=ctx)
    assert e.value.status == -1


@pytest.mark.parametrize("case", ["uniform 3d", "grid ties", "ragged 2d"])
def test_device_plan_equals_oracle(ctx, case):
    """The device plan against the oracle's own tree and traversal (the host
    planner is pinned to the oracle on the CPU; this closes the chain
    directly)."""
    from oracle.tree import build_lists, build_tree
    if case == "uniform 3d":
        pts, leaf, eta = uniform_points(5000, 3, 3), 64, 0.7
    elif case == "grid ties":
        g = np.stack(np.meshgrid(np.arange(16.0), np.arange(16.0)), 0).reshape(2, -1)
        pts, leaf, eta = np.ascontiguousarray(g), 4, 0.7
    else:
        pts, leaf, eta = uniform_points(3001, 2, 8), 37, 1.5
    _say(f"device plan vs oracle: {case}")
    pd = h2.plan_create(pts, leaf, eta, ctx=ctx)
    tr = build_tree(pts, leaf)
    L = build_lists(tr, eta)
    D = int(pd.export("DEPTH")[0])
    assert D == tr.depth
    np.testing.assert_array_equal(pd.export("PERM"), tr.perm)
    nodes = pd.export("NODES").reshape(-1, 2)
    np.testing.assert_array_equal(nodes[:, 0], tr.begin)
    np.testing.assert_array_equal(nodes[:, 1], tr.end)
    boxes = pd.export("BOXES").reshape(-1, 2, pts.shape[0])
    np.testing.assert_array_equal(boxes[:, 0], tr.lo)
    np.testing.assert_array_equal(boxes[:, 1], tr.hi)
    np.testing.assert_array_equal(pd.export("NEAR_PTR"), L.near_ptr)
    np.testing.assert_array_equal(pd.export("NEAR_IDX"), L.near_idx)
    for t in range(D + 1):
        np.testing.assert_array_equal(pd.export("FAR_PTR", t), L.far_ptr[t])
        np.testing.assert_array_equal(pd.export("FAR_IDX", t), L.far_idx[t])
