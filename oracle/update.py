"""Two-sided construction for non-symmetric matrices, and the low-rank update
of an existing H^2 matrix (TEST INFRASTRUCTURE ONLY, like the whole package).

The paper builds symmetric matrices and notes that the non-symmetric case
follows the same steps (Sec. II-A, Sec. III).  Reading used here:
  * Row bases come from Y = A Omega, column bases from Z = A^T Omega', with
    Omega' drawn like Omega from a second seed.  Both sides run the steps of
    Alg. 1 level by level, in lockstep.
  * Each side's random vectors are carried up by the OTHER side's IDs: for an
    admissible pair A(I_s, I_b) ~= U_s B_{s,b} V_b^T, so the far contribution to
    the row samples of the skeleton rows is B_{s,b} (V_b^T Omega_b), and to the
    column samples B_{b,s}^T (U_b^T Omega'_b).
      row side   : Y_loc = Y - sum_{b in N} D_{tau,b} Omega_b        (leaf)
                   Y_loc = [Y_nu - sum_{b in F_nu} B_{nu,b} Omega^c_b]  (inner)
                   Y_next = Y_loc(J_r, :),  Omega^c_next = V^T Omega^c
      column side: Z_loc = Z - sum_{b in N} D_{b,tau}^T Omega'_b
                   Z_loc = [Z_nu - sum_{b in F_nu} B_{b,nu}^T Omega'^r_b]
                   Z_next = Z_loc(J_c, :),  Omega'^r_next = U^T Omega'^r
  * One sample count d for both sides: a level is converged when every cluster
    of both sides is (Sec. III-B test); otherwise d_inc columns of Omega AND of
    Omega' are drawn and swept up.  The threshold delta is the one of the
    symmetric construction, from the norm estimate of the row sketch Y_0.
  * Couplings B_{s,b} = A(I~r_s, I~c_b) (k_r x k_c), near blocks D = A(I_s, I_b).
For a symmetric A with Omega' = Omega the column side repeats the row side
operation by operation, and the result is the symmetric construction.

The update application: A = K_H + U V^T for an H^2 matrix K_H on the same
points and partition.  The sketch is the H^2 matvec plus the low-rank product;
entries come from the H^2 format itself (``H2Matrix.entries``).
"""
from __future__ import annotations

import numpy as np

from .build import SampleLimitError, absolute_threshold, converged, top_depth
from .h2 import H2Matrix
from .linalg import row_id
from .philox import gaussian
from .tree import build_lists, build_tree


class LowRankUpdateOperator:
    """A = K_H + U V^T in original point order (U, V: n x r)."""

    symmetric = False

    def __init__(self, h_old: H2Matrix, U: np.ndarray, V: np.ndarray):
        self.h, self.U, self.V = h_old, np.asarray(U, np.float64), np.asarray(V, np.float64)
        self.n = h_old.tree.n

    def sketch(self, omega):
        return self.h.matvec(omega) + self.U @ (self.V.T @ omega)

    def sketch_t(self, omega):
        return self.h.matvec_t(omega) + self.V @ (self.U.T @ omega)

    def entries(self, rows, cols):
        rows, cols = np.asarray(rows), np.asarray(cols)
        return self.h.entries(rows, cols) + self.U[rows] @ self.V[cols].T

    def dense(self):
        return self.h.dense() + self.U @ self.V.T


class _Side:
    """State of one side (row or column) of the two-sided construction."""

    def __init__(self):
        self.J, self.Umat = {}, {}
        self.om_out, self.y_out = {}, {}


class _TwoSidedBuilder:
    def __init__(self, op, points, leaf_size, eta, tol, d0, d_inc, d_max, seed, seed_c, norm_mode, oversample=0):
        self.op = op
        self.oversample = oversample
        self.tree = build_tree(points, leaf_size)
        self.lists = build_lists(self.tree, eta)
        self.tol, self.d0, self.d_inc, self.d_max = tol, d0, d_inc, d_max
        self.seed, self.seed_c, self.norm_mode = seed, seed_c, norm_mode
        self.h = H2Matrix(self.tree, self.lists)
        self.h.Uc, self.h.Ec, self.h.skel_c = {}, {}, {}
        self.r, self.c = _Side(), _Side()
        self.d = 0

    def draw(self, col0, ncols):
        """Omega, Y = A Omega, Omega', Z = A^T Omega' for columns [col0, col0+ncols), tree order."""
        perm = self.tree.perm
        om = gaussian(self.seed, perm, col0, ncols)
        omc = gaussian(self.seed_c, perm, col0, ncols)
        o1 = np.empty_like(om)
        o1[perm] = om
        o2 = np.empty_like(omc)
        o2[perm] = omc
        return om, self.op.sketch(o1)[perm], omc, self.op.sketch_t(o2)[perm]

    def entries_tree(self, pos_rows, pos_cols):
        perm = self.tree.perm
        return self.op.entries(perm[pos_rows], perm[pos_cols])

    def _rank(self, side, t, i):
        return self.h.rank(t, i) if side is self.r else self.h.rank_c(t, i)

    def _near(self, side, s, b):
        blk = self.h.Dn[(s, b)] if side is self.r else np.ascontiguousarray(self.h.Dn[(b, s)].T)
        return blk

    def _far(self, side, t, s, b):
        return self.h.B[(t, s, b)] if side is self.r else np.ascontiguousarray(self.h.B[(t, b, s)].T)

    def level_inputs(self, t, om_leaf, y_leaf, om_child, y_child):
        D = self.tree.depth
        om, y = [], []
        for i in range(1 << t):
            if t == D:
                r = self.h.rows(D, i)
                om.append(om_leaf[r])
                y.append(y_leaf[r])
            else:
                om.append(np.vstack([om_child[2 * i], om_child[2 * i + 1]]))
                y.append(np.vstack([y_child[2 * i], y_child[2 * i + 1]]))
        return om, y

    def subtract(self, side, t, y_in, om_leaf_rows, om_child_out):
        D = self.tree.depth
        out = []
        if t == D:
            npp, ni = self.lists.near_ptr, self.lists.near_idx
            for s in range(1 << D):
                acc = y_in[s].copy()
                for j in range(npp[s], npp[s + 1]):
                    b = int(ni[j])
                    acc -= self._near(side, s, b) @ om_leaf_rows[b]
                out.append(acc)
            return out
        fp, fi = self.lists.far_ptr[t + 1], self.lists.far_idx[t + 1]
        for i in range(1 << t):
            parts = []
            k1 = self._rank(side, t + 1, 2 * i)
            for nu, part in ((2 * i, y_in[i][:k1]), (2 * i + 1, y_in[i][k1:])):
                acc = part.copy()
                for j in range(fp[nu], fp[nu + 1]):
                    b = int(fi[j])
                    acc -= self._far(side, t + 1, nu, b) @ om_child_out[b]
                parts.append(acc)
            out.append(np.vstack(parts))
        return out

    def shrink_up(self, side, t, yloc, om_in):
        """Y_loc(J, :) with this side's ID; Omega carried up by the OTHER side's ID."""
        other = self.c if side is self.r else self.r
        y_o, om_o = [], []
        for i in range(1 << t):
            y_o.append(yloc[i][side.J[(t, i)]])
            om_o.append(other.Umat[(t, i)].T @ om_in[i])
        return y_o, om_o

    def _sweep_level(self, t, om_new, y_new, omc_new, z_new, child):
        """Inputs and Y_loc of both sides at depth t for one column block."""
        res = {}
        for side, om_l, y_l in ((self.r, om_new, y_new), (self.c, omc_new, z_new)):
            com, cy = child.get(id(side), (None, None))
            om_in, y_in = self.level_inputs(t, om_l, y_l, com, cy)
            yloc = self.subtract(side, t, y_in, om_in, com)
            res[id(side)] = (om_in, yloc)
        return res

    def update_samples(self, t_cur):
        D = self.tree.depth
        if self.d + self.d_inc > self.d_max:
            raise SampleLimitError(f"not converged with d_max={self.d_max} samples")
        om_new, y_new, omc_new, z_new = self.draw(self.d, self.d_inc)
        self.d += self.d_inc
        child = {}
        for t in range(D, t_cur - 1, -1):
            res = self._sweep_level(t, om_new, y_new, omc_new, z_new, child)
            if t == t_cur:
                return res
            child = {}
            for side in (self.r, self.c):
                om_in, yloc = res[id(side)]
                cy, com = self.shrink_up(side, t, yloc, om_in)
                child[id(side)] = (com, cy)
                for i in range(1 << t):
                    side.om_out[t][i] = np.hstack([side.om_out[t][i], com[i]])
                    side.y_out[t][i] = np.hstack([side.y_out[t][i], cy[i]])
        raise AssertionError("unreachable")

    def run(self) -> H2Matrix:
        tr, h = self.tree, self.h
        D = tr.depth
        npp, ni = self.lists.near_ptr, self.lists.near_idx
        for s in range(1 << D):
            for j in range(npp[s], npp[s + 1]):
                b = int(ni[j])
                h.Dn[(s, b)] = self.entries_tree(h.rows(D, s), h.rows(D, b))
        h.top = top_depth(self.lists, D)
        if h.top > D:
            return h
        om0, y0, omc0, z0 = self.draw(0, self.d0)
        self.d = self.d0
        h.delta = absolute_threshold(y0, self.d0, self.tol, 1 << D, self.norm_mode)
        child = {}
        for t in range(D, h.top - 1, -1):
            res = self._sweep_level(t, om0, y0, omc0, z0, child)
            rounds = 0
            while not all(converged(yl, h.delta, self.oversample)
                          for side in (self.r, self.c) for yl in res[id(side)][1]):
                more = self.update_samples(t)
                for side in (self.r, self.c):
                    om_in, yloc = res[id(side)]
                    om_b, yloc_b = more[id(side)]
                    res[id(side)] = ([np.hstack([a, b]) for a, b in zip(om_in, om_b)],
                                     [np.hstack([a, b]) for a, b in zip(yloc, yloc_b)])
                rounds += 1
            h.rounds[t] = rounds
            # IDs of both sides (batchedID)
            for side, Ud, Ed, sk in ((self.r, h.U, h.E, h.skel), (self.c, h.Uc, h.Ec, h.skel_c)):
                yloc = res[id(side)][1]
                for i in range(1 << t):
                    J, U = row_id(yloc[i], h.delta)
                    side.J[(t, i)], side.Umat[(t, i)] = J, U
                    if t == D:
                        Ud[i] = U
                        sk[(t, i)] = h.rows(D, i)[J]
                    else:
                        k1 = len(sk[(t + 1, 2 * i)])
                        Ed[(t + 1, 2 * i)] = U[:k1]
                        Ed[(t + 1, 2 * i + 1)] = U[k1:]
                        rows_bar = np.concatenate([sk[(t + 1, 2 * i)], sk[(t + 1, 2 * i + 1)]])
                        sk[(t, i)] = rows_bar[J]
            child = {}
            for side in (self.r, self.c):
                om_in, yloc = res[id(side)]
                cy, com = self.shrink_up(side, t, yloc, om_in)
                child[id(side)] = (com, cy)
                side.om_out[t], side.y_out[t] = list(com), list(cy)
            # couplings B_{s,b} = A(I~r_s, I~c_b)
            fp, fi = self.lists.far_ptr[t], self.lists.far_idx[t]
            for s in range(1 << t):
                for j in range(fp[s], fp[s + 1]):
                    b = int(fi[j])
                    h.B[(t, s, b)] = self.entries_tree(h.skel[(t, s)], h.skel_c[(t, b)])
        h.samples = self.d
        return h


def build_h2_two_sided(op, points: np.ndarray, leaf_size: int = 64, eta: float = 0.7, tol: float = 1e-6,
                       d0: int = 32, d_inc: int = 16, d_max: int = 1024, seed: int = 1000,
                       seed_c: int | None = None, norm_mode: str = "fro_scaled", oversample: int = 0) -> H2Matrix:
    """Two-sided Alg. 1 + adaptive sampling for a non-symmetric ``op`` (needs
    op.sketch, op.sketch_t and op.entries).  seed_c defaults to seed + 1."""
    sc = seed + 1 if seed_c is None else seed_c
    return _TwoSidedBuilder(op, points, leaf_size, eta, tol, d0, d_inc, d_max, seed, sc, norm_mode,
                            oversample).run()


def update_h2(h_old: H2Matrix, points: np.ndarray, U: np.ndarray, V: np.ndarray, leaf_size: int = 64,
              eta: float = 0.7, tol: float = 1e-6, d0: int = 32, d_inc: int = 16, d_max: int = 1024,
              seed: int = 1002, seed_c: int | None = None, norm_mode: str = "fro_scaled",
              oversample: int = 0) -> H2Matrix:
    """H^2 approximation of K_H + U V^T, built two-sided from the H^2 black box on
    the partition of ``h_old`` (same points, leaf size and eta)."""
    op = LowRankUpdateOperator(h_old, U, V)
    b = _TwoSidedBuilder(op, points, leaf_size, eta, tol, d0, d_inc, d_max, seed,
                         seed + 1 if seed_c is None else seed_c, norm_mode, oversample)
    if not (np.array_equal(b.tree.perm, h_old.tree.perm)
            and all(np.array_equal(a, c) for a, c in zip(b.lists.far_idx, h_old.lists.far_idx))):
        raise ValueError("h_old was built on another partition")
    return b.run()
