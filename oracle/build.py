"""Algorithm 1 with adaptive sampling (Sec. III-A, III-B), symmetric case.

Levels are numbered as in Alg. 1: level 1 is the leaf depth D, level l works on
the clusters at depth D - l + 1, and the root (depth 0) is never processed.

For every processed cluster tau the algorithm keeps
  Omega^l_tau -- the transformed random vectors of its rows  (m_tau x d)
  Y^l_tau     -- the samples of its rows                      (m_tau x d)
where at the leaves the rows are the cluster's points and at an inner cluster
they are the skeletons of its two children, stacked (Alg. 1 merge step).
One level does:
  1. subtract the part already represented at this level (Alg. 1):
       leaf : Y_loc = Y^1_tau - sum_{b in N_tau} D_{tau,b} Omega^1_b, D_{tau,b} = K(I_tau, I_b)
       inner: Y_loc = Y^l_tau - [sum_{b in F_nu1} B_{nu1,b} Omega^l_b ; sum_{b in F_nu2} B_{nu2,b} Omega^l_b]
  2. adaptive test (Sec. III-B; skipped with a fixed sample size, d_inc = 0,
     which takes the d0 columns as they are, Sec. III-A): a cluster is
     converged when the smallest |R_ii|
     of the unpivoted QR of the leading d - p columns of Y_loc is below the
     absolute threshold delta, or when m_tau + p <= d (p = oversampling margin,
     see ``converged``).  While some cluster is not converged, d_inc new columns are drawn,
     sketched and swept up through the levels already finished with the stored
     factors (updateSamples), then appended to Y_loc and Omega^l of this level.
  3. row ID of Y_loc (Sec. II-B):  Y_loc ~= U Y_loc(J, :)   (leaf U_tau, or the
     stacked transfer matrices [E_nu1; E_nu2] at an inner cluster), skeleton
     I~_tau = rows(tau)[J];  Y^{l+1}_tau = Y_loc(J, :);  Omega^{l+1}_tau = U^T Omega^l_tau
     (eq. Yl: the samples of the transformed matrix need only these sub-vectors).
  4. coupling matrices B_{tau,b} = K(I~_tau, I~_b) for b in F_tau.
Levels run from the leaves up to the coarsest depth that holds an admissible
block (``top_depth``); nothing above it is processed.

Readings (the paper leaves these open):
  * absolute threshold: delta = tol * nu / sqrt(#leaves) with
    nu = ||Y_0||_F / sqrt(d0), an unbiased estimate of ||K||_F from the first
    sketch ("an approximate norm of the matrix ... via sketching", Sec. III-B);
    ``norm_mode="literal"`` uses delta = tol * nu.  The same delta is used at every
    level ("ID with eps_l").
  * sample block sizes: d0 initial columns, d_inc per adaptive round; exceeding
    d_max raises.
"""
from __future__ import annotations

import math

import numpy as np

from .h2 import H2Matrix
from .linalg import qr_r_diag, row_id
from .philox import gaussian
from .tree import build_lists, build_tree


class SampleLimitError(RuntimeError):
    pass


def absolute_threshold(Y0: np.ndarray, d0: int, tol: float, n_leaves: int, norm_mode: str) -> float:
    nu = float(np.linalg.norm(Y0)) / math.sqrt(d0)
    if norm_mode == "fro_scaled":
        return tol * nu / math.sqrt(n_leaves)
    if norm_mode == "literal":
        return tol * nu
    raise ValueError(norm_mode)


def top_depth(lists, D: int) -> int:
    """Coarsest depth that holds an admissible block (D + 1 when there is none).

    Reading: levels above it are not processed.  Their IDs would only build
    bases and transfer matrices that no coupling block uses, and their samples
    hold nothing but the truncation residue of the levels below.
    """
    for t in range(1, D + 1):
        if len(lists.far_idx[t]) > 0:
            return t
    return D + 1


def converged(Yloc: np.ndarray, delta: float, oversample: int = 0) -> bool:
    """Adaptive convergence test of one cluster (Sec. III-B): the samples suffice
    when the QR of Y_loc shows a diagonal entry below delta.

    Reading: the test looks only at the leading d - p columns, keeping p
    samples of oversampling (the margin of the fixed-rank scheme, Sec. III-A)
    for the ID: the trailing diagonal entries of a nearly square Gaussian
    sketch are small even for a full-rank block, and without the margin such a
    block is truncated wrongly.  A cluster with m + p <= d has all its rows
    resolved and is converged."""
    m, d = Yloc.shape
    if m + oversample <= d:
        return True
    q = d - oversample
    if q <= 0:
        return False
    return bool(qr_r_diag(Yloc[:, :q]).min() < delta)


class _Builder:
    def __init__(self, op, points, leaf_size, eta, tol, d0, d_inc, d_max, seed, norm_mode, oversample=0):
        self.op = op
        self.oversample = oversample
        self.tree = build_tree(points, leaf_size)
        self.lists = build_lists(self.tree, eta)
        self.tol, self.d0, self.d_inc, self.d_max = tol, d0, d_inc, d_max
        self.seed, self.norm_mode = seed, norm_mode
        self.h = H2Matrix(self.tree, self.lists)
        self.d = 0
        # per-depth state: om_in[t][i], om_out[t][i], y_out[t][i]
        self.om_in, self.om_out, self.y_out = {}, {}, {}

    # -- black box in original order, tree-ordered in/out
    def draw(self, col0: int, ncols: int):
        tr = self.tree
        om_tree = gaussian(self.seed, tr.perm, col0, ncols)     # row p <-> original perm[p]
        om_orig = np.empty_like(om_tree)
        om_orig[tr.perm] = om_tree
        y_tree = self.op.sketch(om_orig)[tr.perm]
        return om_tree, y_tree

    def entries_tree(self, pos_rows, pos_cols):
        perm = self.tree.perm
        return self.op.entries(perm[pos_rows], perm[pos_cols])

    # -- step 1 for one column block at depth t
    def level_inputs(self, t, om_leaf, y_leaf, om_child_out, y_child_out):
        """Omega^l_tau and Y^l_tau of every cluster at depth t (leaf rows or merged children)."""
        D = self.tree.depth
        om, y = [], []
        for i in range(1 << t):
            if t == D:
                r = self.h.rows(D, i)
                om.append(om_leaf[r])
                y.append(y_leaf[r])
            else:
                om.append(np.vstack([om_child_out[2 * i], om_child_out[2 * i + 1]]))
                y.append(np.vstack([y_child_out[2 * i], y_child_out[2 * i + 1]]))
        return om, y

    def subtract(self, t, y_in, om_in_leaf, om_child_out):
        """Y_loc of every cluster at depth t (Alg. 1 batchedBSRGemm step)."""
        D = self.tree.depth
        out = []
        if t == D:
            npp, ni = self.lists.near_ptr, self.lists.near_idx
            for s in range(1 << D):
                acc = y_in[s].copy()
                for j in range(npp[s], npp[s + 1]):
                    b = int(ni[j])
                    acc -= self.h.Dn[(s, b)] @ om_in_leaf[b]
                out.append(acc)
            return out
        fp, fi = self.lists.far_ptr[t + 1], self.lists.far_idx[t + 1]
        for i in range(1 << t):
            parts = []
            for nu in (2 * i, 2 * i + 1):
                k_nu = self.h.rank(t + 1, nu)
                acc = y_in[i][:k_nu].copy() if nu == 2 * i else y_in[i][y_in[i].shape[0] - k_nu:].copy()
                for j in range(fp[nu], fp[nu + 1]):
                    b = int(fi[j])
                    acc -= self.h.B[(t + 1, nu, b)] @ om_child_out[b]
                parts.append(acc)
            out.append(np.vstack(parts))
        return out

    def shrink_up(self, t, yloc, om_in):
        """Step 3 applied with the stored ID of depth t: (Y_loc(J,:), U^T Omega^l)."""
        y_o, om_o = [], []
        for i in range(1 << t):
            J, U = self.J[(t, i)], self.Umat[(t, i)]
            y_o.append(yloc[i][J])
            om_o.append(U.T @ om_in[i])
        return y_o, om_o

    def update_samples(self, t_cur):
        """Draw d_inc new columns and sweep them up to depth t_cur (updateSamples)."""
        D = self.tree.depth
        if self.d + self.d_inc > self.d_max:
            raise SampleLimitError(f"not converged with d_max={self.d_max} samples")
        om_new, y_new = self.draw(self.d, self.d_inc)
        self.d += self.d_inc
        child_om = child_y = None
        for t in range(D, t_cur - 1, -1):
            om_in, y_in = self.level_inputs(t, om_new, y_new, child_om, child_y)
            yloc = self.subtract(t, y_in, om_in, child_om)
            if t == t_cur:
                return om_in, yloc
            child_y, child_om = self.shrink_up(t, yloc, om_in)
            for i in range(1 << t):  # keep the stored upswept vectors complete
                self.om_out[t][i] = np.hstack([self.om_out[t][i], child_om[i]])
                self.y_out[t][i] = np.hstack([self.y_out[t][i], child_y[i]])
        raise AssertionError("unreachable")

    def run(self) -> H2Matrix:
        tr, h = self.tree, self.h
        D = tr.depth
        perm = tr.perm
        # dense near-field blocks D_{tau,b} = K(I_tau, I_b)   (batchedGen)
        npp, ni = self.lists.near_ptr, self.lists.near_idx
        for s in range(1 << D):
            for j in range(npp[s], npp[s + 1]):
                b = int(ni[j])
                h.Dn[(s, b)] = self.entries_tree(h.rows(D, s), h.rows(D, b))
        h.top = top_depth(self.lists, D)
        if h.top > D:      # no admissible block anywhere: the matrix is all dense blocks
            return h
        # Alg. 1: Y = K_blk(Omega)
        om0, y0 = self.draw(0, self.d0)
        self.d = self.d0
        h.delta = absolute_threshold(y0, self.d0, self.tol, 1 << D, self.norm_mode)
        self.J, self.Umat = {}, {}
        child_om = child_y = None
        for t in range(D, h.top - 1, -1):
            om_in, y_in = self.level_inputs(t, om0, y0, child_om, child_y)
            yloc = self.subtract(t, y_in, om_in, child_om)
            rounds = 0
            while self.d_inc > 0 and not all(converged(yl, h.delta, self.oversample) for yl in yloc):
                om_b, yloc_b = self.update_samples(t)
                om_in = [np.hstack([a, b]) for a, b in zip(om_in, om_b)]
                yloc = [np.hstack([a, b]) for a, b in zip(yloc, yloc_b)]
                rounds += 1
            h.rounds[t] = rounds
            # row ID per cluster (batchedID), shrink and upsweep
            for i in range(1 << t):
                J, U = row_id(yloc[i], h.delta)
                self.J[(t, i)], self.Umat[(t, i)] = J, U
                if t == D:
                    h.U[i] = U
                    h.skel[(t, i)] = h.rows(D, i)[J]
                else:
                    k1 = h.rank(t + 1, 2 * i)
                    h.E[(t + 1, 2 * i)] = U[:k1]
                    h.E[(t + 1, 2 * i + 1)] = U[k1:]
                    rows_bar = np.concatenate([h.skel[(t + 1, 2 * i)], h.skel[(t + 1, 2 * i + 1)]])
                    h.skel[(t, i)] = rows_bar[J]
            child_y, child_om = self.shrink_up(t, yloc, om_in)
            self.om_in[t] = om_in
            self.om_out[t], self.y_out[t] = list(child_om), list(child_y)
            # coupling matrices B_{tau,b} = K(I~_tau, I~_b)   (batchedGen)
            fp, fi = self.lists.far_ptr[t], self.lists.far_idx[t]
            for s in range(1 << t):
                for j in range(fp[s], fp[s + 1]):
                    b = int(fi[j])
                    h.B[(t, s, b)] = self.entries_tree(h.skel[(t, s)], h.skel[(t, b)])
        h.samples = self.d
        return h


def build_h2(op, points: np.ndarray, leaf_size: int = 64, eta: float = 0.7, tol: float = 1e-6,
             d0: int = 32, d_inc: int = 16, d_max: int = 1024, seed: int = 1000,
             norm_mode: str = "fro_scaled", oversample: int = 0) -> H2Matrix:
    """Build the H^2 matrix of ``op`` on ``points`` (dim, n) with Alg. 1 + adaptive sampling."""
    return _Builder(op, points, leaf_size, eta, tol, d0, d_inc, d_max, seed, norm_mode, oversample).run()
