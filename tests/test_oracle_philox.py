"""Pins of the oracle's counter-based Gaussian generator (Omega of Alg. 1)."""
import numpy as np
import pytest

from oracle.philox import gaussian, philox4x64_10


def _numpy_philox_block(ctr, key):
    """Philox4x64-10 of counter ``ctr`` from NumPy's own bit generator.

    NumPy increments its counter before each 4-word block, so it is started one
    below the wanted counter (with borrow across the 256-bit counter)."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(ctr)) - 1
    v %= 1 << 256
    start = [(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(start, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 11, 13), (17, 19)),
    ((2**64 - 1, 3, 2**63, 9), (2**64 - 5, 12345)),
    ((123456, 31, 0, 0), (1001, 0)),
])
def test_philox_matches_numpy_bit_generator(ctr, key):
    ours = philox4x64_10(tuple(np.array([c], dtype=np.uint64) for c in ctr), key)
    assert [int(w[0]) for w in ours] == _numpy_philox_block(ctr, key)


def test_gaussian_is_counter_indexed():
    rows = np.array([7, 3, 1000, 5])
    a = gaussian(42, rows, 0, 8)
    b = gaussian(42, rows[::-1], 2, 6)
    # entry (i, j) depends on (seed, i, j) only, not on row order or column block
    np.testing.assert_array_equal(a[::-1, 2:], b)
    assert not np.array_equal(gaussian(43, rows, 0, 8), a)


def test_gaussian_moments():
    z = gaussian(1000, np.arange(200000), 0, 2).ravel()
    assert abs(z.mean()) < 5e-3
    assert abs(z.var() - 1.0) < 1e-2
    # fourth moment of N(0,1) is 3
    assert abs(np.mean(z ** 4) - 3.0) < 0.05
    # tail mass beyond 2 sigma ~ 4.55%
    assert abs(np.mean(np.abs(z) > 2.0) - 0.0455) < 3e-3
