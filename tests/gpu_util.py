"""Shared helpers of the GPU tests: logging, host/device conversion, and the
element-by-element comparison of a built matrix with the oracle's.

Not a test module (no test_ prefix); imported by the tests/test_gpu_*.py files.
"""
from __future__ import annotations

import sys

import numpy as np


def say(msg):
    """Names the case before any GPU work, so a failing run shows which case it was."""
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def to_np(t):
    return t.detach().cpu().numpy()


def colmajor_from(a):
    """(n, c) host array -> (n, c) column-major cuda view (transpose of a contiguous (c, n) tensor)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).cuda().T


def dense_from_matvec(H, n, trans=False):
    import torch
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    return to_np(H.matvec(eye.T.contiguous().T, trans=trans))


def fill_entry_batch(batch, f):
    """Fills an h2_entry_fn block batch on the device: out[off[b] + r + c*rcnt[b]] =
    f(idx[rbeg[b] + r], idx[cbeg[b] + c]), with f evaluated elementwise on
    index tensors (original point indices)."""
    import torch
    nb = batch.nblocks
    rc = batch.rcnt.long()
    sizes = rc * batch.ccnt.long()
    total = int(sizes.sum().item())
    if total == 0:
        return
    blk = torch.repeat_interleave(torch.arange(nb, device="cuda"), sizes)
    start = torch.cumsum(sizes, 0) - sizes
    local = torch.arange(total, device="cuda") - start[blk]
    r = local % rc[blk]
    c = local // rc[blk]
    i = batch.idx[batch.rbeg[blk] + r].long()
    j = batch.idx[batch.cbeg[blk] + c].long()
    batch.out[batch.off[blk] + local] = f(i, j)


def oracle_level_parts(ho, t, col=False):
    """The oracle's factors at depth t in the layout h2_export uses:
    ranks, skeleton original indices, BASIS (node by node, m x k column-major;
    inner nodes [E_nu1; E_nu2]) and COUPLING (far pairs in CSR order, k_s x k_b
    column-major)."""
    D = ho.tree.depth
    perm = ho.tree.perm
    skel = ho.skel_c if (col and ho.two_sided) else ho.skel
    U = ho.Uc if (col and ho.two_sided) else ho.U
    E = ho.Ec if (col and ho.two_sided) else ho.E
    n_t = 1 << t
    ranks = np.array([len(skel.get((t, i), ())) for i in range(n_t)], dtype=np.int32)
    sk = [perm[np.asarray(skel[(t, i)], dtype=np.int64)] for i in range(n_t)]
    bases = []
    for i in range(n_t):
        if t == D:
            Ui = U[i]
        else:
            Ui = np.vstack([E[(t + 1, 2 * i)], E[(t + 1, 2 * i + 1)]])
        bases.append(Ui)
    fp, fi = ho.lists.far_ptr[t], ho.lists.far_idx[t]
    blocks = [ho.B[(t, s, int(fi[j]))] for s in range(n_t) for j in range(fp[s], fp[s + 1])]
    return ranks, sk, bases, blocks


def _split(flat, shapes):
    out, off = [], 0
    for (m, k) in shapes:
        out.append(flat[off:off + m * k].reshape(k, m).T)
        off += m * k
    assert off == flat.size
    return out


EPS = 2.0 ** -53


def id_matrix_bar(H):
    """Bar for the ID matrices U = P^T [I; T^T] against the oracle's, relative to
    each node's largest entry.  The two constructions' samples differ by
    summation-order rounding (a few units of u = 2^-53 of a column's norm); the
    triangular solve T = R11^-1 R12 amplifies that by cond(R11), and the
    truncation keeps |R_kk| >= delta while ||R11|| <~ nu (the norm estimate), so
    cond(R11) <~ nu / delta (= sqrt(#leaves) / tol for the default threshold).
    The factor 100 covers the sqrt(k), sqrt(d) and upper-level growth of that
    estimate (measured: 2-5 u nu / delta)."""
    info = H.info()
    return 100.0 * EPS * info["norm_estimate"] / info["delta"]


def compare_with_oracle(H, ho, col=False, dense=True, block_atol=None):
    """Compares a built matrix with the oracle's construction of the same problem
    (same points, operator, Omega, options).  Structure must be identical: top
    depth, ranks and skeleton sets (both constructions see the same samples up
    to rounding).  Coupling and dense blocks are kernel/operator entries at the
    same indices (entry rounding only: rtol 1e-12 / 1e-13; an operator whose
    entries carry their own differences, such as two H^2 matrices built by the
    two sides, passes block_atol, relative to each block's largest entry).  The
    ID matrices must agree within id_matrix_bar(H) of each node's largest
    entry.  Returns the largest node-relative ID difference per depth."""
    D = ho.tree.depth
    assert int(H.export("TOP")[0]) == ho.top, "top depth"
    sfx = "_C" if col else ""
    basis_diff = {}
    for t in range(ho.top, D + 1):
        ranks_o, sk_o, bases_o, blocks_o = oracle_level_parts(ho, t, col)
        ranks_g = H.export("RANKS" + sfx, t)
        np.testing.assert_array_equal(ranks_g, ranks_o, err_msg=f"ranks at depth {t}")
        skel_g = H.export("SKEL" + sfx, t)
        np.testing.assert_array_equal(skel_g, np.concatenate(sk_o) if sk_o else skel_g[:0],
                                      err_msg=f"skeletons at depth {t}")
        bases_g = _split(H.export("BASIS" + sfx, t), [b.shape for b in bases_o])
        worst = 0.0
        for bg, bo in zip(bases_g, bases_o):
            if bo.size:
                worst = max(worst, float(np.abs(bg - bo).max() / max(np.abs(bo).max(), 1e-300)))
        basis_diff[t] = worst
        if not col:
            blocks_g = _split(H.export("COUPLING", t), [b.shape for b in blocks_o])
            for bg, bo in zip(blocks_g, blocks_o):
                scale = max(np.abs(bo).max(), 1e-300) if bo.size else 1.0
                if block_atol is None:
                    np.testing.assert_allclose(bg, bo, rtol=1e-12, atol=1e-14 * scale)
                else:
                    np.testing.assert_allclose(bg, bo, rtol=0, atol=block_atol * scale)
    if dense and not col:
        Dg = H.export("DENSE")
        off = 0
        npp, ni = ho.lists.near_ptr, ho.lists.near_idx
        for s in range(1 << D):
            for j in range(npp[s], npp[s + 1]):
                ref = ho.Dn[(s, int(ni[j]))]
                got = Dg[off:off + ref.size].reshape(ref.shape[1], ref.shape[0]).T
                np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15 * max(np.abs(ref).max(), 1e-300))
                off += ref.size
        assert off == Dg.size
    if basis_diff:
        bar = id_matrix_bar(H)
        assert max(basis_diff.values()) <= bar, (basis_diff, bar)
    return basis_diff
