"""The H^2 matrix produced by Alg. 1, its matvec and its dense reconstruction.

Representation (Sec. II-A, Table I, nested basis eq.):
  * leaf bases U_tau (m_tau x k_tau), stored explicitly;
  * transfer matrices E_nu (k_nu x k_parent) for every node below depth 1, so an
    inner basis is U_tau = diag(U_nu1, U_nu2) [E_nu1; E_nu2];
  * coupling matrices B_{s,t} (k_s x k_t) for t in F_s at every depth;
  * dense blocks D_{s,t} (m_s x m_t) for t in N_s at the leaf depth.
The matrix is symmetric, so the column basis of a block equals the row basis of
its column cluster: K(I_s, I_t) ~= U_s B_{s,t} U_t^T for an admissible pair.
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

    # ----------------------------------------------------------------- helpers
    def rows(self, depth: int, local: int) -> np.ndarray:
        node = (1 << depth) - 1 + local
        return np.arange(self.tree.begin[node], self.tree.end[node])

    def rank(self, depth: int, local: int) -> int:
        return len(self.skel.get((depth, local), ()))

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
            xh = {D: [self.U[i].T @ X[self.rows(D, i)] for i in range(1 << D)]}
            for t in range(D - 1, top - 1, -1):
                xh[t] = [self.E[(t + 1, 2 * i)].T @ xh[t + 1][2 * i]
                         + self.E[(t + 1, 2 * i + 1)].T @ xh[t + 1][2 * i + 1]
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

    # ---------------------------------------------------------- reconstruction
    def basis(self, depth: int, local: int) -> np.ndarray:
        """Explicit nested basis U_tau (eq. nested_basis) of a node (m_tau x k_tau)."""
        D = self.tree.depth
        if depth == D:
            return self.U[local]
        u1 = self.basis(depth + 1, 2 * local)
        u2 = self.basis(depth + 1, 2 * local + 1)
        top = u1 @ self.E[(depth + 1, 2 * local)]
        bot = u2 @ self.E[(depth + 1, 2 * local + 1)]
        return np.vstack([top, bot])

    def dense(self) -> np.ndarray:
        """K_H as a dense array in ORIGINAL order (small n only)."""
        tr = self.tree
        D = tr.depth
        K = np.zeros((tr.n, tr.n))
        for t in range(self.top, D + 1):
            fp, fi = self.lists.far_ptr[t], self.lists.far_idx[t]
            bases = [self.basis(t, i) for i in range(1 << t)]
            for s in range(1 << t):
                for j in range(fp[s], fp[s + 1]):
                    b = int(fi[j])
                    rs, rb = self.rows(t, s), self.rows(t, b)
                    K[np.ix_(rs, rb)] = bases[s] @ self.B[(t, s, b)] @ bases[b].T
        npp, ni = self.lists.near_ptr, self.lists.near_idx
        for s in range(1 << D):
            for j in range(npp[s], npp[s + 1]):
                b = int(ni[j])
                K[np.ix_(self.rows(D, s), self.rows(D, b))] = self.Dn[(s, b)]
        out = np.empty_like(K)
        out[np.ix_(tr.perm, tr.perm)] = K
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
