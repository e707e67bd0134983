"""Cluster tree, admissibility and dual-tree traversal (Sec. II-A, Figs. 1-3).

Readings of points the paper leaves open (the paper says only "KD-tree, leaf
size 64-256" and "bounding boxes"):
  * Tree: binary KD bisection.  A node's box is the tight axis-aligned box of its
    points.  Split axis = the widest box extent (lowest axis on ties).  The
    node's indices are stably sorted by (coordinate on that axis, original
    index); the left child takes the first floor(n/2), the right child the rest.
  * Depth D = the smallest d with ceil(N / 2^d) <= leaf_size, so every leaf sits
    at depth D (Alg. 1 treats "level 1" as one leaf level).  N <= leaf_size gives
    D = 0: the root is the only leaf.
  * Node numbering: heap order, node i has children 2i+1, 2i+2; depth t holds ids
    2^t-1 .. 2^(t+1)-2.  A node owns the contiguous range [begin, end) of the
    permutation ``perm`` (tree position p -> original index perm[p]).
  * Admissibility (general admissibility condition, Sec. II-A):
        adm(s,t)  <=>  (D(s) + D(t)) / 2 <= eta * Dist(s,t)
    with D = box diagonal and Dist = Euclidean gap between the boxes (0 when they
    touch or overlap).  It is evaluated without square roots: with
    a_s = sum_k (hi-lo)_k^2, a_t likewise, c = sum_k gap_k^2 and
    q = 4 eta^2 c - a_s - a_t, the condition is  q >= 0 and 4 a_s a_t <= q^2.
    Touching or overlapping boxes (c = 0) are never admissible.  All sums run
    over axes in order 0..dim-1, each operation rounded separately (no fused
    multiply-add), so the result is reproducible bit for bit.
  * Traversal: pairs of same-depth clusters starting at (root, root); an
    admissible pair is a far block, an inadmissible pair at the leaf depth is a
    dense (near) block, otherwise the four child pairs are visited.  The lists are
    therefore: near N_tau at the leaf depth only, far F_tau at every depth >= 1.
    Both (s,t) and (t,s) appear; each list is sorted ascending.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def tree_depth(n: int, leaf_size: int) -> int:
    """Smallest d with ceil(n / 2^d) <= leaf_size."""
    if leaf_size < 1:
        raise ValueError("leaf_size >= 1")
    d = 0
    while -(-n // (1 << d)) > leaf_size:
        d += 1
    return d


@dataclass
class ClusterTree:
    dim: int
    n: int
    depth: int                 # D: leaves are at depth D
    perm: np.ndarray           # int64 [n]: tree position -> original index
    begin: np.ndarray          # int64 [2^(D+1)-1]
    end: np.ndarray            # int64 [2^(D+1)-1]
    lo: np.ndarray             # float64 [nodes, dim] tight box lower corner
    hi: np.ndarray             # float64 [nodes, dim] tight box upper corner

    @property
    def num_nodes(self) -> int:
        return (1 << (self.depth + 1)) - 1

    def level_nodes(self, t: int) -> range:
        return range((1 << t) - 1, (1 << (t + 1)) - 1)

    def size(self, node: int) -> int:
        return int(self.end[node] - self.begin[node])


def build_tree(points: np.ndarray, leaf_size: int) -> ClusterTree:
    """KD bisection tree of the points (dim, n), following the reading above."""
    dim, n = points.shape
    D = tree_depth(n, leaf_size)
    nn = (1 << (D + 1)) - 1
    perm = np.arange(n, dtype=np.int64)
    begin = np.zeros(nn, dtype=np.int64)
    end = np.zeros(nn, dtype=np.int64)
    lo = np.zeros((nn, dim))
    hi = np.zeros((nn, dim))
    begin[0], end[0] = 0, n
    for node in range(nn):
        b, e = int(begin[node]), int(end[node])
        idx = perm[b:e]
        if e > b:
            lo[node] = points[:, idx].min(axis=1)
            hi[node] = points[:, idx].max(axis=1)
        if 2 * node + 2 < nn:  # inner node: split
            ext = hi[node] - lo[node]
            axis = int(np.argmax(ext))  # first maximum = lowest axis on ties
            order = np.lexsort((idx, points[axis, idx]))  # by coordinate, then original index
            perm[b:e] = idx[order]
            mid = b + (e - b) // 2
            begin[2 * node + 1], end[2 * node + 1] = b, mid
            begin[2 * node + 2], end[2 * node + 2] = mid, e
    return ClusterTree(dim, n, D, perm, begin, end, lo, hi)


def admissible(lo_s, hi_s, lo_t, hi_t, eta: float) -> bool:
    """Square-root-free general admissibility condition (Sec. II-A), scalar form."""
    dim = len(lo_s)
    a_s = 0.0
    a_t = 0.0
    c = 0.0
    for k in range(dim):
        es = float(hi_s[k]) - float(lo_s[k])
        a_s = a_s + es * es
        et = float(hi_t[k]) - float(lo_t[k])
        a_t = a_t + et * et
        g = max(max(0.0, float(lo_t[k]) - float(hi_s[k])), float(lo_s[k]) - float(hi_t[k]))
        c = c + g * g
    if not c > 0.0:
        return False
    q = ((4.0 * (eta * eta)) * c - a_s) - a_t
    return q >= 0.0 and (4.0 * a_s) * a_t <= q * q


def admissible_many(tree: ClusterTree, s: np.ndarray, t: np.ndarray, eta: float) -> np.ndarray:
    """Vectorised form of ``admissible`` over node pairs (same operations, same order)."""
    a_s = np.zeros(s.shape[0])
    a_t = np.zeros(s.shape[0])
    c = np.zeros(s.shape[0])
    for k in range(tree.dim):
        es = tree.hi[s, k] - tree.lo[s, k]
        a_s = a_s + es * es
        et = tree.hi[t, k] - tree.lo[t, k]
        a_t = a_t + et * et
        g = np.maximum(np.maximum(0.0, tree.lo[t, k] - tree.hi[s, k]), tree.lo[s, k] - tree.hi[t, k])
        c = c + g * g
    q = ((4.0 * (eta * eta)) * c - a_s) - a_t
    return (c > 0.0) & (q >= 0.0) & ((4.0 * a_s) * a_t <= q * q)


@dataclass
class Lists:
    """Per-depth CSR interaction lists over LOCAL node indices (node - (2^t - 1))."""
    near_ptr: np.ndarray          # leaf depth only
    near_idx: np.ndarray
    far_ptr: list                 # far_ptr[t], t = 0..D (t = 0 is empty)
    far_idx: list


def _to_csr(rows: np.ndarray, cols: np.ndarray, nrows: int):
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(ptr, rows + 1, 1)
    return np.cumsum(ptr), cols.astype(np.int64)


def build_lists(tree: ClusterTree, eta: float) -> Lists:
    """Dual-tree traversal (Sec. II-A) producing N_tau and F_tau (Table I).

    The traversal is carried out depth by depth: the inadmissible pairs of depth t
    spawn their four child pairs at depth t+1.  The set of pairs visited is the
    same as that of the recursive formulation.
    """
    D = tree.depth
    far_ptr, far_idx = [], []
    s = np.array([0], dtype=np.int64)
    t = np.array([0], dtype=np.int64)
    near_ptr = near_idx = None
    for depth in range(D + 1):
        base = (1 << depth) - 1
        adm = admissible_many(tree, s, t, eta)
        fp, fi = _to_csr(s[adm] - base, t[adm] - base, 1 << depth)
        far_ptr.append(fp)
        far_idx.append(fi)
        s_in, t_in = s[~adm], t[~adm]
        if depth == D:
            near_ptr, near_idx = _to_csr(s_in - base, t_in - base, 1 << depth)
        else:
            cs = np.stack([2 * s_in + 1, 2 * s_in + 1, 2 * s_in + 2, 2 * s_in + 2], axis=1).ravel()
            ct = np.stack([2 * t_in + 1, 2 * t_in + 2, 2 * t_in + 1, 2 * t_in + 2], axis=1).ravel()
            s, t = cs, ct
    return Lists(near_ptr, near_idx, far_ptr, far_idx)


def traverse_recursive(tree: ClusterTree, eta: float):
    """The recursive dual-tree traversal exactly as described in Sec. II-A.

    Returns (near, far) as sets of (depth, s_local, t_local).  Used by the tests
    as an independent derivation of ``build_lists`` on small trees.
    """
    near, far = set(), set()
    D = tree.depth

    def depth_of(node):
        return int(np.floor(np.log2(node + 1)))

    def visit(s, t):
        d = depth_of(s)
        base = (1 << d) - 1
        if admissible(tree.lo[s], tree.hi[s], tree.lo[t], tree.hi[t], eta):
            far.add((d, s - base, t - base))
        elif d == D:
            near.add((d, s - base, t - base))
        else:
            for i in (2 * s + 1, 2 * s + 2):
                for j in (2 * t + 1, 2 * t + 2):
                    visit(i, j)

    visit(0, 0)
    return near, far
