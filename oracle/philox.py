"""Counter-based Gaussian random matrix Omega for the sketch (Alg. 1, batchedRand).

The paper only asks for "a random matrix" (Alg. 1 inputs).  Reading: i.i.d.
standard normal entries, where entry (i, j) -- i the ORIGINAL point index, j the
global sample-column index (columns continue across adaptive rounds) -- is a
pure function of (seed, i, j).  This makes Omega independent of the point
permutation and of any launch shape.

Generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11), written here from that description:
  * state: 4 x 64-bit counter words, 2 x 64-bit key words;
  * one round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (full 128-bit products),
    c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
  * between rounds the key is bumped by the Weyl constants (k0 += W0, k1 += W1);
  * 10 rounds.
Gaussian: Box-Muller on two uniforms in (0,1) built from the top 53 bits of the
first two output words: u = (w >> 11 + 1/2) * 2^-53;  z = sqrt(-2 ln u1) cos(2 pi u2).
Counter = (i, j, 0, 0); key = (seed, 0).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: np.uint64):
    """Full 64x64 -> 128-bit product split into (hi, lo), via 32-bit halves."""
    a = np.asarray(a, dtype=np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2^64
    return hi, lo


def philox4x64_10(ctr, key):
    """Apply Philox4x64-10 to counters ctr (4 arrays of uint64) under key (2 uint64)."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64).copy() for c in ctr)
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = np.uint64((int(k0) + int(W0)) & 0xFFFFFFFFFFFFFFFF)
                k1 = np.uint64((int(k1) + int(W1)) & 0xFFFFFFFFFFFFFFFF)
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _unit_open(w: np.ndarray) -> np.ndarray:
    """Top 53 bits of w mapped to the open interval (0,1): (w>>11 + 0.5) * 2^-53."""
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def gaussian(seed: int, rows: np.ndarray, col0: int, ncols: int) -> np.ndarray:
    """Omega(rows, col0:col0+ncols) as a float64 (len(rows), ncols) array.

    ``rows`` are original point indices.  Entry (i, j) depends only on (seed, i, j).
    """
    rows = np.asarray(rows, dtype=np.uint64)
    n = rows.shape[0]
    ii = np.repeat(rows, ncols)
    jj = np.tile(np.arange(col0, col0 + ncols, dtype=np.uint64), n)
    zero = np.zeros_like(ii)
    w0, w1, _, _ = philox4x64_10((ii, jj, zero, zero), (np.uint64(seed), np.uint64(0)))
    u1 = _unit_open(w0)
    u2 = _unit_open(w1)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos((2.0 * np.pi) * u2)
    return z.reshape(n, ncols)
