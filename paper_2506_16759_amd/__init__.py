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
from ._lib import BF16X3, BF16X6, FP32, FP32E, FP64, K_EXP, K_GAUSS, NORM_FRO_SCALED, NORM_LITERAL, H2Error

__all__ = ["opts_default", "Context", "Plan", "plan_create", "gaussian", "sketch", "build", "build_batched",
           "build_update", "autotune_leaf",
           "H2Matrix",
           "kernel_spec", "H2Error", "K_EXP", "K_GAUSS", "FP64", "FP32", "BF16X3", "FP32E", "BF16X6", "NORM_FRO_SCALED",
           "NORM_LITERAL"]


def _torch():
    import torch
    return torch


def kernel_spec(kind, length: float) -> _lib.Kernel:
    k = {"exp": K_EXP, "gauss": K_GAUSS}.get(kind, kind)
    return _lib.Kernel(int(k), float(length))


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


def _export(fn, handle, name: str, depth: int = 0) -> np.ndarray:
    part = _lib.PART[name]
    need = C.c_size_t(0)
    _lib.check(fn(handle, part, depth, None, 0, C.byref(need)), "export")
    dt = np.dtype(_lib.PART_DTYPE[name])
    out = np.empty(need.value // dt.itemsize, dtype=dt)
    if need.value:
        _lib.check(fn(handle, part, depth, out.ctypes.data_as(C.c_void_p), need.value, C.byref(need)), "export")
    return out


class Plan(_Handle):
    """Host-only cluster tree + interaction lists (h2_plan_*)."""

    _free = "h2_plan_free"

    def __init__(self, points: np.ndarray, leaf_size: int, eta: float):
        self._h = None
        pts = np.ascontiguousarray(points, dtype=np.float64)
        dim, n = pts.shape
        h = C.c_void_p()
        lib = self._lib_ref = _lib.load()
        _lib.check(lib.h2_plan_create(n, dim, pts.ctypes.data_as(C.c_void_p), leaf_size, float(eta), C.byref(h)),
                   "h2_plan_create")
        self._h = h
        self.n, self.dim = n, dim

    def export(self, name: str, depth: int = 0) -> np.ndarray:
        return _export(_lib.load().h2_plan_export, self._h, name, depth)


def plan_create(points: np.ndarray, leaf_size: int = 64, eta: float = 0.7) -> Plan:
    return Plan(points, leaf_size, eta)


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
    k = kernel_spec(kernel, length)
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

    def matvec(self, x):
        """K_H x for x an (n, c) column-major cuda tensor (or an (n,) vector)."""
        vec = x.dim() == 1
        if vec:
            x = x.reshape(1, -1).T
        ldx = _colmajor(x, self.n)
        c = x.shape[1]
        y = empty_colmajor(self.n, c)
        _lib.check(_lib.load().h2_matvec(self.ctx._h, self._h, c, C.c_void_p(x.data_ptr()), ldx,
                                         C.c_void_p(y.data_ptr()), self.n), "h2_matvec")
        return y[:, 0] if vec else y

    def export(self, name: str, depth: int = 0) -> np.ndarray:
        return _export(_lib.load().h2_export, self._h, name, depth)

    def info(self) -> dict:
        inf = _lib.Info()
        _lib.check(_lib.load().h2_query(self._h, C.byref(inf)), "h2_query")
        return inf.as_dict()


def build(ctx: Context, points, kernel="exp", length: float = 0.2, opts: _lib.Opts | None = None,
          **opt_over) -> H2Matrix:
    """Algorithm 1 with adaptive sampling on the GPU (h2_build).  points: (dim, n)."""
    torch = _torch()
    pts = torch.as_tensor(points).to(device="cuda", dtype=torch.float64).contiguous()
    dim, n = pts.shape
    o = opts if opts is not None else opts_default(**opt_over)
    k = kernel_spec(kernel, length)
    h = C.c_void_p()
    _lib.check(_lib.load().h2_build(ctx._h, n, dim, C.c_void_p(pts.data_ptr()), C.byref(k), C.byref(o),
                                    C.byref(h)), "h2_build")
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
        arr[i] = _lib.Problem(n, dim, pts.data_ptr(), kernel_spec(pr.get("kernel", "exp"), pr.get("length", 0.2)),
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


def build_batched(ctx: Context, problems, precision=FP64, d_max: int = 96, use_graph: bool = True,
                  return_info: bool = False, first_pass: int = 0):
    """Many independent constructions in one launch sequence (h2_build_batched).

    problems: sequence of dicts with keys points ((dim, n) array or tensor),
    kernel, length, and optionally tol, leaf_size, eta, d0, d_inc, seed,
    norm_mode, oversample (defaults as h2_opts_default).  first_pass: columns
    of the first launch sequence (0: largest d0 + 32; problems not converged
    within them are built again with d_max).  Returns a list of H2Matrix (and
    the batch info dict when return_info)."""
    if isinstance(precision, str):
        precision = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp32e": FP32E, "bf16x6": BF16X6}[precision]
    arr, keep = _problem_array(problems)
    bo = _lib.BatchOpts(int(precision), int(d_max), 1 if use_graph else 0, int(first_pass))
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
