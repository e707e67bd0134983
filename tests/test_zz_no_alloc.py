"""h2_matvec_noalloc (the product without device allocation, for callers that
cannot allocate) against h2_matvec, through the C ABI: two calls in a row, the
second on a smaller matrix with fewer columns, so a stale scratch array from
the first call would show; both products of a two-sided (updated) matrix; the
rejection of a matrix whose temporaries exceed the scratch array.

Bar: the same kernels on column chunks of another width, so the products agree
to summation-order rounding: |y_noalloc - y| <= 1e-14 max |y| per call.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_16759_amd as h2
from paper_2506_16759_amd import _lib
from paper_2506_16759_amd.workloads import gaussian_factors, uniform_points
from gpu_util import colmajor_from, say, to_np


@pytest.fixture(scope="module")
def ctx():
    return h2.Context(0)


def _compare(H, n, c, seed, trans=False):
    import torch
    x = colmajor_from(np.random.default_rng(seed).standard_normal((n, c)))
    ref = to_np(H.matvec(x, trans=trans))
    y = torch.full((c, n), float("nan"), dtype=torch.float64, device="cuda").T
    H.matvec_noalloc(x, y, trans=trans)
    got = to_np(y)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"n={n} c={c} trans={trans}: max difference {err:.3e} (bitwise equal: {np.array_equal(got, ref)})")
    assert err <= 1e-14
    return got


def test_noalloc_matvec_two_calls(ctx):
    say("no-alloc matvec: 20000-point 3D matrix, 70 columns, then 3000-point 2D matrix, 5 columns")
    p1 = uniform_points(20000, 3, 5)
    H1 = h2.build(ctx, p1, "exp", 0.2, tol=1e-6, leaf_size=64, seed=1)
    _compare(H1, 20000, 70, 1)
    p2 = uniform_points(3000, 2, 6)
    H2 = h2.build(ctx, p2, "gauss", 0.1, tol=1e-7, leaf_size=32, seed=2)
    _compare(H2, 3000, 5, 2)
    _compare(H1, 20000, 1, 3)


def test_noalloc_matvec_two_sided(ctx):
    n = 4000
    say(f"no-alloc matvec of an updated (two-sided) matrix, n={n}")
    pts = uniform_points(n, 3, 7)
    H = h2.build(ctx, pts, "exp", 0.2, tol=1e-6, leaf_size=48, seed=3)
    U, V = gaussian_factors(n, 6, 8)
    Hu = h2.build_update(ctx, H, 10.0 * U, V, tol=1e-6, oversample=5, seed=4)
    _compare(Hu, n, 9, 4)
    _compare(Hu, n, 9, 5, trans=True)


def test_noalloc_matvec_rejects_oversized(ctx):
    import torch
    n = 600_000
    say(f"no-alloc matvec rejects a matrix beyond its scratch array: n={n} (2D, tol 1e-3)")
    pts = uniform_points(n, 2, 9)
    H = h2.build(ctx, pts, "exp", 0.1, tol=1e-3, leaf_size=64, d0=16, d_inc=16, seed=5)
    x = torch.zeros((1, n), dtype=torch.float64, device="cuda").T
    y = torch.zeros((1, n), dtype=torch.float64, device="cuda").T
    with pytest.raises(h2.H2Error) as ei:
        H.matvec_noalloc(x, y)
    assert ei.value.status == -1
    assert "bytes of scratch" in str(ei.value)
    say(f"rejected: {ei.value}")
    H.close()
    # the context is still usable afterwards
    p2 = uniform_points(2000, 3, 10)
    H2 = h2.build(ctx, p2, "exp", 0.2, tol=1e-6, leaf_size=32, seed=6)
    _compare(H2, 2000, 3, 6)
