"""Matrix operators given to the construction (Alg. 1 inputs, Sec. V-A).

Alg. 1 needs two things from the matrix: a black box Y = K Omega and a way to
evaluate any sub-block K(I_s, I_t).  Here both are written out plainly, in
ORIGINAL point order:
  * ``KernelOperator`` -- K(x, y) = kappa(|x - y|) on a point cloud.  The sketch is
    the dense product computed block row by block row; entries are evaluated
    directly.  Kernels (parameter p):
      exp       : exp(-r / p)            exponential covariance, eq. (cov), p = l
      gauss     : exp(-r^2 / (2 p^2))    Gaussian covariance (reading: the usual
                                         squared-exponential form), p = l
      helmholtz : cos(p r) / r           volume-IE operator of the Helmholtz
                                         equation, eq. (ie), p = wavenumber k
    The covariance kernels include the diagonal (x = y): kappa(0) = 1.  The IE
    kernel is defined for x != y only; reading: its diagonal, and any pair of
    coincident points (r = 0), is 0.
  * ``CallbackOperator`` -- user-supplied sketch and entry functions, used for
    the exactly-low-rank checks and for sketching an existing H^2 matrix plus a
    low-rank product.
"""
from __future__ import annotations

import numpy as np


def pair_distance(xa: np.ndarray, xb: np.ndarray) -> np.ndarray:
    """r[i, j] = |xa[:, i] - xb[:, j]| with the squared terms summed over axes in order."""
    r2 = np.zeros((xa.shape[1], xb.shape[1]))
    for a in range(xa.shape[0]):
        diff = xa[a][:, None] - xb[a][None, :]
        r2 = r2 + diff * diff
    return np.sqrt(r2)


def kernel_from_distance(kind: str, param: float, r: np.ndarray) -> np.ndarray:
    """kappa(r) elementwise (Sec. V-A): param is the correlation length l, or the
    wavenumber k of the Helmholtz kernel."""
    if kind == "exp":
        return np.exp(-(r / param))
    if kind == "gauss":
        return np.exp(-(r * r) / (2.0 * param * param))
    if kind == "helmholtz":
        r = np.asarray(r, dtype=np.float64)
        out = np.zeros_like(r)
        pos = r > 0
        out[pos] = np.cos(param * r[pos]) / r[pos]
        return out
    raise ValueError(f"unknown kernel {kind!r}")


class KernelOperator:
    """Dense kernel matrix K(i, j) = kappa(|x_i - x_j|), accessed implicitly."""

    symmetric = True

    def __init__(self, points: np.ndarray, kind: str, param: float, block_rows: int = 256):
        self.points = np.ascontiguousarray(points, dtype=np.float64)
        self.kind = kind
        self.length = float(param)      # correlation length, or the Helmholtz wavenumber
        self.block_rows = block_rows
        self.n = self.points.shape[1]

    def entries(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        """K(rows, cols) for original indices rows, cols."""
        xa = self.points[:, np.asarray(rows, dtype=np.int64)]
        xb = self.points[:, np.asarray(cols, dtype=np.int64)]
        return kernel_from_distance(self.kind, self.length, pair_distance(xa, xb))

    def sketch(self, omega: np.ndarray) -> np.ndarray:
        """Y = K Omega (original order), one block of rows at a time."""
        omega = np.asarray(omega, dtype=np.float64)
        y = np.zeros((self.n, omega.shape[1]))
        allc = np.arange(self.n)
        for r0 in range(0, self.n, self.block_rows):
            rows = np.arange(r0, min(self.n, r0 + self.block_rows))
            y[rows] = self.entries(rows, allc) @ omega
        return y

    def sketch_rows(self, rows: np.ndarray, omega: np.ndarray) -> np.ndarray:
        """(K Omega)(rows, :) only -- used to check sampled rows of a large sketch."""
        rows = np.asarray(rows)
        omega = np.asarray(omega, dtype=np.float64)
        out = np.zeros((rows.shape[0], omega.shape[1]))
        allc = np.arange(self.n)
        for r0 in range(0, rows.shape[0], self.block_rows):
            out[r0:r0 + self.block_rows] = self.entries(rows[r0:r0 + self.block_rows], allc) @ omega
        return out

    sketch_t = sketch

    def dense(self) -> np.ndarray:
        allc = np.arange(self.n)
        return self.entries(allc, allc)


class CallbackOperator:
    """A matrix known only through y = A x (and A^T x) and an entry evaluator."""

    def __init__(self, n: int, sketch, entries, sketch_t=None, symmetric: bool = True):
        self.n = n
        self._sketch = sketch
        self._sketch_t = sketch_t if sketch_t is not None else sketch
        self._entries = entries
        self.symmetric = symmetric

    def sketch(self, omega):
        return np.asarray(self._sketch(np.asarray(omega, dtype=np.float64)), dtype=np.float64)

    def sketch_t(self, omega):
        return np.asarray(self._sketch_t(np.asarray(omega, dtype=np.float64)), dtype=np.float64)

    def entries(self, rows, cols):
        return np.asarray(self._entries(np.asarray(rows), np.asarray(cols)), dtype=np.float64)
