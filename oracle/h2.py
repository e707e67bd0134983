"""The H^2 matrix produced by Alg. 1, its matvec and its dense reconstruction.

Representation (Sec. II-A, Table I, nested basis eq.):
  * leaf bases U_tau (m_tau x k_tau), stored explicitly;
  * transfer matrices E_nu (k_nu x k_parent) for every node below depth 1, so an
    inner basis is U_tau = diag(U_nu1, U_nu2) [E_nu1; E_nu2];
  * coupling matrices B_{s,t} (k_s x k_t) for t in F_s at every depth;
  * dense blocks D_{s,t} (m_s x m_t) for t in N_s at the leaf depth.
A symmetric build uses one basis per cluster: K(I_s, I_t) ~= U_s B_{s,t} U_t^T
for an admissible pair.  A two-sided build (non-symmetric matrix) also holds
column bases V (leaf ``Uc``, transfer ``Ec``, skeletons ``skel_c``), and then
A(I_s, I_t) ~= U_s B_{s,t} V_t^T with B_{s,t} of size k_s x kc_t.
Internally all row indices are tree positions; the public functions take and
return vectors in original point order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .tree import ClusterTree, Lists


@dataclass
class H2Matrix:
    tree: ClusterTree
    lists: Lists
    delta: float = 0.0
    top: int = 1                                # coarsest processed depth
    U: dict = field(default_factory=dict)       # leaf local -> (m x k)
    E: dict = field(default_factory=dict)       # (depth, local) -> (k_node x k_parent)
    skel: dict = field(default_factory=dict)    # (depth, local) -> tree positions
    Dn: dict = field(default_factory=dict)      # (s_local, b_local) at leaf depth -> dense
    B: dict = field(default_factory=dict)       # (depth, s_local, b_local) -> coupling
    samples: int = 0                            # total sample columns drawn
    rounds: dict = field(default_factory=dict)  # depth -> adaptive rounds taken there
    Uc: dict | None = None                      # column side of a two-sided build (else None)
    Ec: dict | None = None
    skel_c: dict | None = None

    @property
    def two_sided(self) -> bool:
        return self.Uc is not None

    # ----------------------------------------------------------------- helpers
    def rows(self, depth: int, local: int) -> np.ndarray:
        node = (1 << depth) - 1 + local
        return np.arange(self.tree.begin[node], self.tree.end[node])

    def rank(self, depth: int, local: int) -> int:
        return len(self.skel.get((depth, local), ()))

    def rank_c(self, depth: int, local: int) -> int:
        """Column-side rank (equals the row rank of a symmetric build)."""
        if not self.two_sided:
            return self.rank(depth, local)
        return len(self.skel_c.get((depth, local), ()))

    def ranks(self):
        """{depth: array of ranks} for the processed depths top..D."""
        D = self.tree.depth
        return {t: np.array([self.rank(t, i) for i in range(1 << t)]) for t in range(self.top, D + 1)}

    # ------------------------------------------------------------------ matvec
    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = K_H x for x in original order, shape (n,) or (n, c).

        Standard H^2 product: upsweep x_hat = U^T x (leaves) and
        x_hat_tau = sum E_nu^T x_hat_nu; coupling y_hat_s = sum_{t in F_s} B_{s,t} x_hat_t;
        downsweep y_hat_nu += E_nu y_hat_parent, y = U y_hat; plus the near field.
        """
        tr = self.tree
        vec = x.ndim == 1
        X = x.reshape(tr.n, -1)[tr.perm]              # tree order
        c = X.shape[1]
        D = tr.depth
        Y = np.zeros_like(X)
        if 0 < D and self.top <= D:
            top = self.top
            Uc, Ec = (self.Uc, self.Ec) if self.two_sided else (self.U, self.E)
            xh = {D: [Uc[i].T @ X[self.rows(D, i)] for i in range(1 << D)]}
            for t in range(D - 1, top - 1, -1):
                xh[t] = [Ec[(t + 1, 2 * i)].T @ xh[t + 1][2 * i]
                         + Ec[(t + 1, 2 * i + 1)].T @ xh[t + 1][2 * i + 1]
                         for i in range(1 << t)]
            yh = {}
            for t in range(top, D + 1):
                fp, fi = self.lists.far_ptr[t], self.lists.far_idx[t]
                yh[t] = []
                for s in range(1 << t):
                    acc = np.zeros((self.rank(t, s), c))
                    for j in range(fp[s], fp[s + 1]):
                        b = int(fi[j])
                        acc += self.B[(t, s, b)] @ xh[t][b]
                    yh[t].append(acc)
            for t in range(top + 1, D + 1):
                for i in range(1 << t):
                    yh[t][i] = yh[t][i] + self.E[(t, i)] @ yh[t - 1][i // 2]
            for i in range(1 << D):
                Y[self.rows(D, i)] += self.U[i] @ yh[D][i]
        npp, ni = self.lists.near_ptr, self.lists.near_idx
        for s in range(1 << D):
            for j in range(npp[s], npp[s + 1]):
                b = int(ni[j])
                Y[self.rows(D, s)] += self.Dn[(s, b)] @ X[self.rows(D, b)]
        out = np.empty_like(Y)
        out[tr.perm] = Y
        return out.ravel() if vec else out

    def matvec_t(self, x: np.ndarray) -> np.ndarray:
        """y = K_H^T x (original order).  Symmetric builds: the matvec itself.
        Two-sided: upsweep with the row bases, y_hat_t = sum_{s in F_t} B_{s,t}^T x_hat_s
        (the far lists are symmetric), downsweep with the column bases, near field
        with D_{s,t}^T."""
        if not self.two_sided:
            return self.matvec(x)
        tr = self.tree
        vec = x.ndim == 1
        X = x.reshape(tr.n, -1)[tr.perm]
        c = X.shape[1]
        D = tr.depth
        Y = np.zeros_like(X)
        if 0 < D and self.top <= D:
            top = self.top
            xh = {D: [self.U[i].T @ X[self.rows(D, i)] for i in range(1 << D)]}
            for t in range(D - 1, top - 1, -1):
                xh[t] = [self.E[(t + 1, 2 * i)].T @ xh[t + 1][2 * i]
                         + self.E[(t + 1, 2 * i + 1)].T @ xh[t + 1][2 * i + 1]
                         for i in range(1 << t)]
            yh = {}
            for t in range(top, D + 1):
                fp, fi = self.lists.far_ptr[t], self.lists.far_idx[t]
                yh[t] = [np.zeros((self.rank_c(t, u), c)) for u in range(1 << t)]
                for s in range(1 << t):
                    for j in range(fp[s], fp[s + 1]):
                        u = int(fi[j])
                        yh[t][u] += self.B[(t, s, u)].T @ xh[t][s]
            for t in range(top + 1, D + 1):
                for i in range(1 << t):
                    yh[t][i] = yh[t][i] + self.Ec[(t, i)] @ yh[t - 1][i // 2]
            for i in range(1 << D):
                Y[self.rows(D, i)] += self.Uc[i] @ yh[D][i]
        npp, ni = self.lists.near_ptr, self.lists.near_idx
        for s in range(1 << D):
            for j in range(npp[s], npp[s + 1]):
                b = int(ni[j])
                Y[self.rows(D, b)] += self.Dn[(s, b)].T @ X[self.rows(D, s)]
        out = np.empty_like(Y)
        out[tr.perm] = Y
        return out.ravel() if vec else out

    # ---------------------------------------------------------- reconstruction
    def basis(self, depth: int, local: int, col: bool = False) -> np.ndarray:
        """Explicit nested basis U_tau (eq. nested_basis) of a node (m_tau x k_tau);
        col=True gives the column basis V_tau of a two-sided build."""
        D = self.tree.depth
        U, E = (self.Uc, self.Ec) if (col and self.two_sided) else (self.U, self.E)
        if depth == D:
            return U[local]
        u1 = self.basis(depth + 1, 2 * local, col)
        u2 = self.basis(depth + 1, 2 * local + 1, col)
        top = u1 @ E[(depth + 1, 2 * local)]
        bot = u2 @ E[(depth + 1, 2 * local + 1)]
        return np.vstack([top, bot])

    def dense(self) -> np.ndarray:
        """K_H as a dense array in ORIGINAL order (small n only)."""
        tr = self.tree
        D = tr.depth
        K = np.zeros((tr.n, tr.n))
        for t in range(self.top, D + 1):
            fp, fi = self.lists.far_ptr[t], self.lists.far_idx[t]
            bases = [self.basis(t, i) for i in range(1 << t)]
            cbases = [self.basis(t, i, col=True) for i in range(1 << t)] if self.two_sided else bases
            for s in range(1 << t):
                for j in range(fp[s], fp[s + 1]):
                    b = int(fi[j])
                    rs, rb = self.rows(t, s), self.rows(t, b)
                    K[np.ix_(rs, rb)] = bases[s] @ self.B[(t, s, b)] @ cbases[b].T
        npp, ni = self.lists.near_ptr, self.lists.near_idx
        for s in range(1 << D):
            for j in range(npp[s], npp[s + 1]):
                b = int(ni[j])
                K[np.ix_(self.rows(D, s), self.rows(D, b))] = self.Dn[(s, b)]
        out = np.empty_like(K)
        out[np.ix_(tr.perm, tr.perm)] = K
        return out

    def entries(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        """K_H(rows, cols) for original indices, from the definition of the format:
        the entry (i, j) belongs to exactly one block of the partition -- a dense
        leaf block D_{s,t}, or the admissible pair (s, t) of clusters containing
        i and j, where it equals row_i(U_s) B_{s,t} row_j(V_t)^T with the nested
        bases written out (eq. nested_basis).  Rows and columns are grouped by
        leaf so every block is visited once."""
        tr = self.tree
        D = tr.depth
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        inv = np.empty(tr.n, dtype=np.int64)
        inv[tr.perm] = np.arange(tr.n)
        pr, pc = inv[rows], inv[cols]
        first_leaf = (1 << D) - 1
        leaf_begin = tr.begin[first_leaf:first_leaf + (1 << D)]
        lr = np.searchsorted(leaf_begin, pr, side="right") - 1
        lc = np.searchsorted(leaf_begin, pc, side="right") - 1
        out = np.zeros((rows.size, cols.size))
        if getattr(self, "_blocks", None) is None:   # lookup tables, built once per matrix
            near = {(s, int(b)) for s in range(1 << D)
                    for b in self.lists.near_idx[self.lists.near_ptr[s]:self.lists.near_ptr[s + 1]]}
            far = set()
            for t in range(1, D + 1):
                fp, fi = self.lists.far_ptr[t], self.lists.far_idx[t]
                for s in range(1 << t):
                    for j in range(fp[s], fp[s + 1]):
                        far.add((t, s, int(fi[j])))
            self._blocks = (near, far, {})
        near, far, bases = self._blocks

        def basis_rows(t, s, pos, col):
            key = (t, s, col)
            if key not in bases:
                bases[key] = self.basis(t, s, col)
            node = (1 << t) - 1 + s
            return bases[key][pos - tr.begin[node]]

        for a in np.unique(lr):
            ia = np.nonzero(lr == a)[0]
            for b in np.unique(lc):
                jb = np.nonzero(lc == b)[0]
                if (int(a), int(b)) in near:
                    node_a, node_b = first_leaf + a, first_leaf + b
                    blk = self.Dn[(int(a), int(b))]
                    out[np.ix_(ia, jb)] = blk[np.ix_(pr[ia] - tr.begin[node_a], pc[jb] - tr.begin[node_b])]
                    continue
                for t in range(D, 0, -1):
                    s, u = int(a) >> (D - t), int(b) >> (D - t)
                    if (t, s, u) in far:
                        Ur = basis_rows(t, s, pr[ia], False)
                        Vc = basis_rows(t, u, pc[jb], True)
                        out[np.ix_(ia, jb)] = Ur @ self.B[(t, s, u)] @ Vc.T
                        break
                else:
                    raise AssertionError("pair not covered by the partition")
        return out

    def storage_entries(self) -> dict:
        """Number of stored floating-point entries by kind."""
        return {
            "U": sum(u.size for u in self.U.values()),
            "E": sum(e.size for e in self.E.values()),
            "B": sum(b.size for b in self.B.values()),
            "D": sum(d.size for d in self.Dn.values()),
        }


def relative_fro_error(K: np.ndarray, KH: np.ndarray) -> float:
    return float(np.linalg.norm(K - KH) / np.linalg.norm(K))


def power_method_error(apply_diff, apply_ref, n: int, iters: int = 20, seed: int = 7) -> float:
    """Relative 2-norm error by power iteration (Sec. V-A: "a few iterations of the
    power method" on the difference between the H^2 matrix and the sampler).

    apply_diff(x) = (K_H - K) x, apply_ref(x) = K x; both symmetric operators.
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    y = rng.standard_normal(n)
    nd = nr = 0.0
    for _ in range(iters):
        x = x / np.linalg.norm(x)
        x = apply_diff(x)
        nd = np.linalg.norm(x)
        y = y / np.linalg.norm(y)
        y = apply_ref(y)
        nr = np.linalg.norm(y)
    return float(nd / nr)
