"""Householder QR, column-pivoted QR and the interpolative decomposition.

  * ``qr_r_diag``  -- unpivoted Householder QR, returning |R_ii|.  The adaptive
    convergence test (Sec. III-B) looks at the smallest absolute diagonal entry
    of the triangular factor of a node's samples.
  * ``cpqr``       -- column-pivoted Householder QR A P = Q R (Sec. II-B), with
    the column-norm downdating of Businger-Golub and the recompute safeguard of
    Drmac-Bujanovic (as in LAPACK's xLAQP2): a downdated norm is recomputed
    exactly once it has lost about half of its digits.  Pivot = largest
    remaining norm; ties go to the lowest original column index.  Truncation
    (reading of "discarding R_3 when its norm becomes small enough"): stop at the
    first step j whose pivot norm |R_jj| is below the absolute threshold delta,
    so the rank is k = j.  delta = 0 runs to min(rows, cols) steps.
  * ``column_id`` -- A ~= A(:, S) [I T] P^T with T = R_1^{-1} R_2 by back
    substitution (Sec. II-B, ID equation).
  * ``row_id`` -- the row ID used by Alg. 1: rows J of Y reproduce Y through
    Y ~= U Y(J,:), where U (m x k) carries the identity on rows J and T^T on the
    other rows (U = [T I]^T up to the row permutation, Sec. III-A).
"""
from __future__ import annotations

import math

import numpy as np

_EPS = np.finfo(np.float64).eps
_TOL3Z = math.sqrt(_EPS)


def _house(x: np.ndarray):
    """Householder vector v (v[0] = 1) and scalar tau with (I - tau v v^T) x = beta e1."""
    alpha = x[0]
    sigma = float(np.dot(x[1:], x[1:]))
    v = x.copy()
    v[0] = 1.0
    if sigma == 0.0:
        # already a multiple of e1: no reflection needed
        v[1:] = 0.0
        return v, 0.0, alpha
    norm = math.sqrt(alpha * alpha + sigma)
    beta = -norm if alpha >= 0.0 else norm
    v[1:] = x[1:] / (alpha - beta)
    tau = (beta - alpha) / beta
    return v, tau, beta


def qr_r_diag(Y: np.ndarray) -> np.ndarray:
    """|R_ii|, i < min(m, d), of the unpivoted Householder QR of Y (m x d)."""
    A = np.array(Y, dtype=np.float64, copy=True)
    m, d = A.shape
    out = np.zeros(min(m, d))
    for j in range(min(m, d)):
        v, tau, beta = _house(A[j:, j])
        out[j] = abs(beta)
        if tau != 0.0 and j + 1 < d:
            w = v @ A[j:, j + 1:]
            A[j:, j + 1:] -= tau * np.outer(v, w)
    return out


def cpqr(A: np.ndarray, delta: float = 0.0):
    """Column-pivoted Householder QR of A (rows x cols), truncated at |R_jj| < delta.

    Returns (k, piv, R) where piv is the full column permutation (piv[j] is the
    original index of the column moved to position j) and R (min(rows,cols) x
    cols) holds the computed triangular factor in pivoted column order; only its
    first k rows are meaningful after truncation.
    """
    A = np.array(A, dtype=np.float64, copy=True)
    rows, cols = A.shape
    piv = np.arange(cols)
    vn1 = np.sqrt(np.sum(A * A, axis=0))      # partial column norms
    vn2 = vn1.copy()                           # norms at the last exact computation
    steps = min(rows, cols)
    k = steps
    for j in range(steps):
        # pivot: largest partial norm among positions j..cols-1, ties -> lowest original index
        cand = vn1[j:]
        best = cand.max()
        ties = np.nonzero(cand == best)[0] + j
        p = int(ties[np.argmin(piv[ties])])
        if p != j:
            A[:, [j, p]] = A[:, [p, j]]
            piv[[j, p]] = piv[[p, j]]
            vn1[[j, p]] = vn1[[p, j]]
            vn2[[j, p]] = vn2[[p, j]]
        v, tau, beta = _house(A[j:, j])
        if abs(beta) < delta:
            k = j
            break
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        if tau != 0.0 and j + 1 < cols:
            w = v @ A[j:, j + 1:]
            A[j:, j + 1:] -= tau * np.outer(v, w)
        # downdate the remaining norms: n_c <- n_c * sqrt(1 - (R_jc / n_c)^2), or
        # recompute n_c exactly when it has fallen below sqrt(eps) of its last exact value
        c = np.arange(j + 1, cols)
        c = c[vn1[c] != 0.0]
        if c.size:
            t = np.abs(A[j, c]) / vn1[c]
            t = np.maximum(0.0, 1.0 - t * t)
            t2 = t * (vn1[c] / vn2[c]) ** 2
            redo = t2 <= _TOL3Z
            keep = c[~redo]
            vn1[keep] = vn1[keep] * np.sqrt(t[~redo])
            again = c[redo]
            if again.size:
                vn1[again] = np.linalg.norm(A[j + 1:, again], axis=0) if j + 1 < rows else 0.0
                vn2[again] = vn1[again]
    R = np.triu(A[:steps, :])
    return k, piv, R


def back_substitute(R11: np.ndarray, R12: np.ndarray) -> np.ndarray:
    """T = R11^{-1} R12 for upper-triangular R11 (k x k), column by column."""
    k = R11.shape[0]
    T = np.array(R12, dtype=np.float64, copy=True)
    for i in range(k - 1, -1, -1):
        if i + 1 < k:
            T[i, :] -= R11[i, i + 1:] @ T[i + 1:, :]
        T[i, :] /= R11[i, i]
    return T


def column_id(A: np.ndarray, delta: float):
    """Column ID A ~= A(:, S) [I T] P^T (Sec. II-B).  Returns (S, T, piv, k)."""
    k, piv, R = cpqr(A, delta)
    T = back_substitute(R[:k, :k], R[:k, k:])
    return piv[:k].copy(), T, piv, k


def row_id(Y: np.ndarray, delta: float):
    """Row ID of the samples Y (m x d): Y ~= U Y(J, :), via the column ID of Y^T.

    Returns (J, U): J (k,) the skeleton rows in pivot order, U (m x k) with
    U[J[i], :] = e_i exactly and U[piv[k + r], :] = T[:, r]^T.
    """
    m = Y.shape[0]
    J, T, piv, k = column_id(Y.T, delta)
    U = np.zeros((m, k))
    U[J, np.arange(k)] = 1.0
    if k < m:
        U[piv[k:], :] = T.T
    return J, U
