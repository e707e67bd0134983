"""Python binding of libh2, the MI355X H^2 construction library (include/h2.h).

Argument marshalling only: every step of the construction runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory and the stream.
Column-major (n x c) device matrices are represented by the transpose view of
a C-contiguous (c, n) torch tensor, so ``t.data_ptr()`` is the column-major
buffer with leading dimension n.

The library is loaded lazily; importing this package needs neither the GPU nor
the built library (``workloads`` and ``plan_create`` work on any host).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (BF16X3, BF16X6, FP32, FP32E, FP64, FP64_SYM, K_EXP, K_GAUSS, K_HELMHOLTZ, NORM_FRO_SCALED, NORM_LITERAL,
                   H2Error)

__all__ = ["opts_default", "Context", "Plan", "plan_create", "gaussian", "sketch", "build", "build_batched",
           "build_update", "autotune_leaf", "autotune_tiles", "device_view", "EntryBatch",
           "H2Matrix",
           "kernel_spec", "H2Error", "K_EXP", "K_GAUSS", "K_HELMHOLTZ", "FP64", "FP32", "BF16X3", "FP32E", "BF16X6",
           "FP64_SYM", "NORM_FRO_SCALED", "NORM_LITERAL"]


def _torch():
    import torch
    return torch


def kernel_spec(kind, length: float = 0.0, wavenumber: float | None = None) -> _lib.Kernel:
    """h2_kernel for "exp" / "gauss" (correlation length) or "helmholtz" (wavenumber k,
    taken from ``wavenumber``, else from the second argument)."""
    k = {"exp": K_EXP, "gauss": K_GAUSS, "helmholtz": K_HELMHOLTZ}.get(kind, kind)
    if int(k) == K_HELMHOLTZ:
        return _lib.Kernel(int(k), 0.0, float(length if wavenumber is None else wavenumber))
    return _lib.Kernel(int(k), float(length), 0.0)


def opts_default(**over) -> _lib.Opts:
    o = _lib.Opts()
    _lib.check(_lib.load().h2_opts_default(C.byref(o)), "h2_opts_default")
    for k, v in over.items():
        if k == "norm_mode" and isinstance(v, str):
            v = {"fro_scaled": NORM_FRO_SCALED, "literal": NORM_LITERAL}[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp32e": FP32E, "bf16x6": BF16X6}[v]
        setattr(o, k, v)
    return o


class _Handle:
    """Owner of one library handle, freed through the library object it was
    created with: close() reads nothing but the instance, since module globals
    may already be gone when it runs at interpreter exit."""

    _free = ""
    _h = None
    _lib_ref = None

    def close(self):
        h, lib = self._h, self._lib_ref
        self._h = None
        if h and lib is not None:
            getattr(lib, self._free)(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _export(fn, handle, name: str, depth: int = 0, device: bool = False):
    """A part as a NumPy array, or (device=True, h2_export only) as a cuda tensor."""
    part = _lib.PART[name]
    need = C.c_size_t(0)
    dev = (1,) if device else ((0,) if fn is _lib.load().h2_export else ())
    _lib.check(fn(handle, part, depth, *dev, None, 0, C.byref(need)), "export")
    dt = np.dtype(_lib.PART_DTYPE[name])
    if device:
        torch = _torch()
        out = torch.empty(need.value // dt.itemsize, dtype=torch.float64 if dt.kind == "f" else torch.int32,
                          device="cuda")
        ptr = out.data_ptr()
    else:
        out = np.empty(need.value // dt.itemsize, dtype=dt)
        ptr = out.ctypes.data
    if need.value:
        _lib.check(fn(handle, part, depth, *dev, C.c_void_p(ptr), need.value, C.byref(need)), "export")
    return out


class _CudaArray:
    """__cuda_array_interface__ of memory the library hands to a callback."""

    def __init__(self, ptr: int, shape, typestr: str, strides=None):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                         "strides": strides, "version": 2}


def device_view(ptr: int, shape, dtype="f8", ld: int | None = None):
    """A torch cuda tensor aliasing device memory at ptr (no copy): 1-D of length
    shape[0], or 2-D column-major (rows, cols) with leading dimension ld."""
    torch = _torch()
    typestr = {"f8": "<f8", "i4": "<i4", "i8": "<i8"}[dtype]
    item = int(typestr[-1])
    if len(shape) == 1 or shape[0] * shape[-1] == 0:
        obj = _CudaArray(ptr, shape, typestr)
    else:
        rows, cols = shape
        obj = _CudaArray(ptr, (rows, cols), typestr, (item, item * (ld if ld is not None else rows)))
    return torch.as_tensor(obj, device="cuda")


class EntryBatch:
    """Arguments of an entry callback (h2_entry_fn) as device tensors.

    Block b is A(idx[rbeg[b] : rbeg[b] + rcnt[b]], idx[cbeg[b] : cbeg[b] + ccnt[b]]),
    written column-major at out[off[b]:].  Original point indices."""

    def __init__(self, nblocks, idx, rbeg, rcnt, cbeg, ccnt, off, out, max_rows, max_cols):
        self.nblocks, self.max_rows, self.max_cols = int(nblocks), int(max_rows), int(max_cols)
        nb = self.nblocks
        self.rbeg = device_view(rbeg, (nb,), "i8")
        self.rcnt = device_view(rcnt, (nb,), "i4")
        self.cbeg = device_view(cbeg, (nb,), "i8")
        self.ccnt = device_view(ccnt, (nb,), "i4")
        self.off = device_view(off, (nb,), "i8")
        nidx = int(max((self.rbeg + self.rcnt).max().item(), (self.cbeg + self.ccnt).max().item()))
        nout = int((self.off + self.rcnt.long() * self.ccnt.long()).max().item())
        self.idx = device_view(idx, (nidx,), "i4")
        self.out = device_view(out, (nout,), "f8")
        self._ptrs = (idx, rbeg, rcnt, cbeg, ccnt, off, out)

    def blocks(self):
        """Host list of (row indices, column indices, out offset) per block."""
        idx = self.idx.cpu().numpy()
        rb, rc = self.rbeg.cpu().numpy(), self.rcnt.cpu().numpy()
        cb, cc = self.cbeg.cpu().numpy(), self.ccnt.cpu().numpy()
        off = self.off.cpu().numpy()
        return [(idx[rb[b]:rb[b] + rc[b]], idx[cb[b]:cb[b] + cc[b]], int(off[b])) for b in range(self.nblocks)]


class Plan(_Handle):
    """Cluster tree + interaction lists (h2_plan_*): built on the host, or by
    device kernels when a Context is given (h2_plan_create_device; points may
    then be a device tensor)."""

    _free = "h2_plan_free"

    def __init__(self, points, leaf_size: int, eta: float, ctx: "Context | None" = None):
        self._h = None
        h = C.c_void_p()
        lib = self._lib_ref = _lib.load()
        if ctx is None:
            pts = np.ascontiguousarray(points, dtype=np.float64)
            dim, n = pts.shape
            _lib.check(lib.h2_plan_create(n, dim, pts.ctypes.data_as(C.c_void_p), leaf_size, float(eta),
                                          C.byref(h)), "h2_plan_create")
        else:
            torch = _torch()
            pts = torch.as_tensor(points).to(device=f"cuda:{ctx.device}", dtype=torch.float64).contiguous()
            dim, n = pts.shape
            _lib.check(lib.h2_plan_create_device(ctx._h, n, dim, C.c_void_p(pts.data_ptr()), leaf_size,
                                                 float(eta), C.byref(h)), "h2_plan_create_device")
        self._h = h
        self.n, self.dim = n, dim

    def export(self, name: str, depth: int = 0) -> np.ndarray:
        return _export(_lib.load().h2_plan_export, self._h, name, depth)


def plan_create(points, leaf_size: int = 64, eta: float = 0.7, ctx: "Context | None" = None) -> Plan:
    """h2_plan_create (host), or h2_plan_create_device when ctx is given."""
    return Plan(points, leaf_size, eta, ctx)


class Context(_Handle):
    """h2_ctx bound to a device and (by default) torch's current stream."""

    _free = "h2_ctx_destroy"

    def __init__(self, device: int = 0, stream=None):
        self._h = None
        self._lib_ref = _lib.load()
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library needs an MI355X")
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        _lib.check(_lib.load().h2_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)), "h2_ctx_create")
        self._h = h

    def synchronize(self):
        self.stream.synchronize()


def _colmajor(t, rows: int):
    """Check that t is a (rows, c) view of a contiguous (c, rows) float64 cuda tensor."""
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 cuda tensor")
    if t.dim() != 2 or t.shape[0] != rows:
        raise ValueError("expected an (n, c) tensor")
    if t.shape[1] <= 1:             # a single column: its stride is irrelevant
        if t.stride(0) != 1 and rows > 1:
            raise ValueError("expected unit row stride")
        return max(rows, 1)
    if t.stride(0) != 1 or t.stride(1) < rows:
        raise ValueError("expected an (n, c) column-major view (the transpose of a contiguous (c, n) tensor)")
    return t.stride(1)


def empty_colmajor(n: int, c: int, device="cuda"):
    return _torch().empty((c, n), dtype=_torch().float64, device=device).T


def gaussian(ctx: Context, seed: int, rows, col0: int, ncols: int):
    """Omega(rows, col0:col0+ncols) as an (len(rows), ncols) column-major tensor (h2_gaussian)."""
    torch = _torch()
    rows = rows.to(device="cuda", dtype=torch.int32).contiguous()
    n = rows.numel()
    out = empty_colmajor(n, ncols)
    _lib.check(_lib.load().h2_gaussian(ctx._h, seed, n, C.c_void_p(rows.data_ptr()), col0, ncols,
                                       C.c_void_p(out.data_ptr()), max(n, 1)), "h2_gaussian")
    return out


def sketch(ctx: Context, points, kernel, length: float, omega, precision: int = FP64):
    """Y = K(points, points) Omega with the fused on-the-fly kernel (h2_sketch)."""
    torch = _torch()
    pts = points.to(device="cuda", dtype=torch.float64).contiguous()
    dim, n = pts.shape
    ldo = _colmajor(omega, n)
    nc = omega.shape[1]
    y = empty_colmajor(n, nc)
    k = kernel_spec(kernel, length)  # for "helmholtz", length is the wavenumber
    _lib.check(_lib.load().h2_sketch(ctx._h, n, dim, C.c_void_p(pts.data_ptr()), C.byref(k), precision, nc,
                                     C.c_void_p(omega.data_ptr()), ldo, C.c_void_p(y.data_ptr()), max(n, 1)),
               "h2_sketch")
    return y


class H2Matrix(_Handle):
    """A built H^2 matrix (h2_matrix): matvec, export, query."""

    _free = "h2_free"

    def __init__(self, ctx: Context, handle, n: int):
        self.ctx, self._h, self.n = ctx, handle, n
        self._lib_ref = _lib.load()

    def matvec(self, x, trans: bool = False):
        """A_H x (or A_H^T x) for x an (n, c) column-major cuda tensor (or an (n,) vector)."""
        vec = x.dim() == 1
        if vec:
            x = x.reshape(1, -1).T
        ldx = _colmajor(x, self.n)
        c = x.shape[1]
        y = empty_colmajor(self.n, c)
        _lib.check(_lib.load().h2_matvec(self.ctx._h, self._h, 1 if trans else 0, c, C.c_void_p(x.data_ptr()), ldx,
                                         C.c_void_p(y.data_ptr()), self.n), "h2_matvec")
        return y[:, 0] if vec else y

    def matvec_noalloc(self, x, y, trans: bool = False):
        """y = A_H x (or A_H^T x) through h2_matvec_noalloc, which allocates no
        device memory: x and y are (n, c) column-major cuda tensors the caller
        allocated (y is overwritten)."""
        ldx = _colmajor(x, self.n)
        ldy = _colmajor(y, self.n)
        if x.shape[1] != y.shape[1]:
            raise ValueError("x and y must have the same number of columns")
        _lib.check(_lib.load().h2_matvec_noalloc(self.ctx._h, self._h, 1 if trans else 0, x.shape[1],
                                                 C.c_void_p(x.data_ptr()), ldx, C.c_void_p(y.data_ptr()), ldy),
                   "h2_matvec_noalloc")
        return y

    def entries_raw(self, nblocks, idx, rbeg, rcnt, cbeg, ccnt, off, out, max_rows, max_cols):
        """h2_entries on raw device pointers (the entry-callback argument list)."""
        _lib.check(_lib.load().h2_entries(self.ctx._h, self._h, nblocks, *(C.c_void_p(p) for p in
                                                                           (idx, rbeg, rcnt, cbeg, ccnt, off, out)),
                                          max_rows, max_cols), "h2_entries")

    def entries(self, rows, cols):
        """A_H(rows, cols) for original indices (one block), as a (len(rows), len(cols)) cuda tensor."""
        torch = _torch()
        r = torch.as_tensor(np.asarray(rows), dtype=torch.int32)
        c = torch.as_tensor(np.asarray(cols), dtype=torch.int32)
        idx = torch.cat([r, c]).cuda()
        z = lambda v, dt: torch.tensor([v], dtype=dt, device="cuda")
        rb, rc, cb, cc, off = (z(0, torch.int64), z(r.numel(), torch.int32), z(r.numel(), torch.int64),
                               z(c.numel(), torch.int32), z(0, torch.int64))
        out = empty_colmajor(r.numel(), c.numel())
        if r.numel() and c.numel():
            self.entries_raw(1, idx.data_ptr(), rb.data_ptr(), rc.data_ptr(), cb.data_ptr(), cc.data_ptr(),
                             off.data_ptr(), out.data_ptr(), r.numel(), c.numel())
        return out

    def export(self, name: str, depth: int = 0, device: bool = False):
        return _export(_lib.load().h2_export, self._h, name, depth, device)

    def info(self) -> dict:
        inf = _lib.Info()
        _lib.check(_lib.load().h2_query(self._h, C.byref(inf)), "h2_query")
        return inf.as_dict()


def _sketch_callback(fn):
    """h2_sketch_fn from an H2Matrix (its product, zero copy) or from a callable
    fn(omega, y) on (n, d) column-major cuda views that writes y = A omega."""
    if isinstance(fn, H2Matrix):
        H = fn

        def raw(user, n, d, om, ldo, y, ldy, stream):
            try:
                _lib.check(_lib.load().h2_matvec(H.ctx._h, H._h, 0, d, C.c_void_p(om), ldo, C.c_void_p(y), ldy),
                           "h2_matvec")
                return 0
            except Exception:   # any failure aborts the build with H2_ERR_CALLBACK
                return 1
    else:
        def raw(user, n, d, om, ldo, y, ldy, stream):
            try:
                fn(device_view(om, (n, d), ld=ldo), device_view(y, (n, d), ld=ldy))
                return 0
            except Exception:
                return 1
    return _lib.SKETCH_FN(raw)


def _entry_callback(fn):
    """h2_entry_fn from an H2Matrix (h2_entries, zero copy) or from a callable
    fn(batch: EntryBatch) that fills batch.out."""
    if isinstance(fn, H2Matrix):
        H = fn

        def raw(user, nb, idx, rb, rc, cb, cc, off, out, mr, mc, stream):
            try:
                H.entries_raw(nb, idx, rb, rc, cb, cc, off, out, mr, mc)
                return 0
            except Exception:
                return 1
    else:
        def raw(user, nb, idx, rb, rc, cb, cc, off, out, mr, mc, stream):
            try:
                fn(EntryBatch(nb, idx, rb, rc, cb, cc, off, out, mr, mc))
                return 0
            except Exception:
                return 1
    return _lib.ENTRY_FN(raw)


def build(ctx: Context, points, kernel="exp", length: float = 0.2, opts: _lib.Opts | None = None,
          sketch=None, entries=None, wavenumber: float | None = None, **opt_over) -> H2Matrix:
    """Algorithm 1 with adaptive sampling on the GPU (h2_build).  points: (dim, n).

    kernel: "exp", "gauss" (correlation length ``length``), "helmholtz"
    (wavenumber ``wavenumber``, else ``length``) or None.  sketch: None (the
    fused kernel sketch), an H2Matrix (its product is the black box) or a
    callable fn(omega, y).  entries (only with kernel=None): an H2Matrix
    (h2_entries) or a callable fn(EntryBatch)."""
    torch = _torch()
    pts = torch.as_tensor(points).to(device="cuda", dtype=torch.float64).contiguous()
    dim, n = pts.shape
    o = opts if opts is not None else opts_default(**opt_over)
    kp = C.byref(kernel_spec(kernel, length, wavenumber)) if kernel is not None else None
    sk = _sketch_callback(sketch) if sketch is not None else _lib.SKETCH_FN()
    en = _entry_callback(entries) if entries is not None else _lib.ENTRY_FN()
    h = C.c_void_p()
    _lib.check(_lib.load().h2_build(ctx._h, n, dim, C.c_void_p(pts.data_ptr()), kp, sk, None, en, None,
                                    C.byref(o), C.byref(h)), "h2_build")
    del sk, en   # the callbacks are not used after the build
    return H2Matrix(ctx, h, n)


def _problem_array(problems):
    torch = _torch()
    d = opts_default()
    arr = (_lib.Problem * len(problems))()
    keep = []
    for i, pr in enumerate(problems):
        pts = torch.as_tensor(pr["points"]).to(device="cuda", dtype=torch.float64).contiguous()
        keep.append(pts)
        dim, n = pts.shape
        nm = pr.get("norm_mode", d.norm_mode)
        if isinstance(nm, str):
            nm = {"fro_scaled": NORM_FRO_SCALED, "literal": NORM_LITERAL}[nm]
        arr[i] = _lib.Problem(n, dim, pts.data_ptr(), kernel_spec(pr.get("kernel", "exp"), pr.get("length", 0.2),
                                                                pr.get("wavenumber")),
                              pr.get("tol", d.tol), pr.get("leaf_size", d.leaf_size), pr.get("eta", d.eta),
                              pr.get("d0", d.d0), pr.get("d_inc", d.d_inc), pr.get("seed", d.seed), nm,
                              pr.get("oversample", d.oversample))
    return arr, keep


def autotune_leaf(ctx: Context, problems, candidates=(32, 64, 128), precision=FP64, d_max: int = 96,
                  first_pass: int = 0):
    """Leaf size per problem from h2_autotune_leaf (problems and options as for build_batched)."""
    if isinstance(precision, str):
        precision = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp32e": FP32E, "bf16x6": BF16X6}[precision]
    arr, keep = _problem_array(problems)
    cand = (C.c_int32 * len(candidates))(*candidates)
    best = (C.c_int32 * len(problems))()
    bo = _lib.BatchOpts(int(precision), int(d_max), 1, int(first_pass))
    _lib.check(_lib.load().h2_autotune_leaf(ctx._h, len(problems), arr, C.byref(bo), cand, len(candidates), best),
               "h2_autotune_leaf")
    del keep
    return [int(b) for b in best]


def autotune_tiles(ctx: Context, problems, precision=FP64, d_max: int = 96, first_pass: int = 0):
    """Tile shapes for this batch from h2_autotune_tiles (problems and options
    as for build_batched).  Returns dict(sketch_cols, bsr_cols, times_ms), the
    device times of the candidates (sketch_cols 64, 48, 32 with bsr_cols 64,
    then bsr_cols 64, 48, 32, 16 with the chosen sketch_cols)."""
    if isinstance(precision, str):
        precision = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp32e": FP32E, "bf16x6": BF16X6}[precision]
    arr, keep = _problem_array(problems)
    bo = _lib.BatchOpts(int(precision), int(d_max), 1, int(first_pass))
    tuned = _lib.BatchOpts()
    times = (C.c_double * 7)()
    _lib.check(_lib.load().h2_autotune_tiles(ctx._h, len(problems), arr, C.byref(bo), C.byref(tuned), times),
               "h2_autotune_tiles")
    del keep
    return {"sketch_cols": int(tuned.sketch_cols), "bsr_cols": int(tuned.bsr_cols), "times_ms": list(times)}


def build_batched(ctx: Context, problems, precision=FP64, d_max: int = 96, use_graph: bool = True,
                  return_info: bool = False, first_pass: int = 0, sketch_cols: int = 0, bsr_cols: int = 0):
    """Many independent constructions in one launch sequence (h2_build_batched).

    problems: sequence of dicts with keys points ((dim, n) array or tensor),
    kernel, length, and optionally tol, leaf_size, eta, d0, d_inc, seed,
    norm_mode, oversample (defaults as h2_opts_default).  first_pass: columns
    of the first launch sequence (0: largest d0 + 32; problems not converged
    within them are built again with d_max).  sketch_cols, bsr_cols: tile
    shapes (0: default; see autotune_tiles).  Returns a list of H2Matrix (and
    the batch info dict when return_info)."""
    if isinstance(precision, str):
        precision = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp32e": FP32E, "bf16x6": BF16X6}[precision]
    arr, keep = _problem_array(problems)
    bo = _lib.BatchOpts(int(precision), int(d_max), 1 if use_graph else 0, int(first_pass), int(sketch_cols),
                        int(bsr_cols))
    handles = (C.c_void_p * len(problems))()
    info = _lib.BatchInfo()
    _lib.check(_lib.load().h2_build_batched(ctx._h, len(problems), arr, C.byref(bo), handles, C.byref(info)),
               "h2_build_batched")
    mats = [H2Matrix(ctx, C.c_void_p(handles[i]), int(arr[i].n)) for i in range(len(problems))]
    return (mats, info.as_dict()) if return_info else mats


def build_update(ctx: Context, old: H2Matrix, U=None, V=None, opts: _lib.Opts | None = None,
                 **opt_over) -> H2Matrix:
    """H^2 approximation of old + U V^T on old's partition (h2_build_update).

    U, V: (n, r) arrays or tensors in original point order (None for r = 0).
    Options as for build (leaf_size and eta come from old); seed keys Omega,
    seed + 1 keys Omega'."""
    torch = _torch()
    o = opts if opts is not None else opts_default(**opt_over)
    n = old.n
    if U is None:
        r, up, vp, keep = 0, None, None, ()
    else:
        Ut = torch.as_tensor(U).to(device="cuda", dtype=torch.float64)
        Vt = torch.as_tensor(V).to(device="cuda", dtype=torch.float64)
        if Ut.shape != Vt.shape or Ut.shape[0] != n:
            raise ValueError("U and V must both be (n, r)")
        r = Ut.shape[1]
        Uc, Vc = Ut.T.contiguous(), Vt.T.contiguous()   # (r, n) C-order = column-major n x r
        up, vp, keep = C.c_void_p(Uc.data_ptr()), C.c_void_p(Vc.data_ptr()), (Uc, Vc)
    h = C.c_void_p()
    _lib.check(_lib.load().h2_build_update(ctx._h, old._h, r, up, n, vp, n, C.byref(o), C.byref(h)),
               "h2_build_update")
    del keep
    return H2Matrix(ctx, h, n)
