"""ctypes declarations of the C ABI in include/h2.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2.so")

H2_OK = 0
STATUS = {0: "H2_OK", -1: "H2_ERR_ARG", -2: "H2_ERR_HIP", -3: "H2_ERR_OOM", -4: "H2_ERR_CALLBACK",
          -5: "H2_ERR_SAMPLES", -6: "H2_ERR_STATE", -7: "H2_ERR_UNSUPPORTED"}

K_EXP, K_GAUSS, K_HELMHOLTZ = 1, 2, 3
FP64, FP32, BF16X3, FP32E, BF16X6, FP64_SYM = 0, 1, 2, 3, 4, 5
NORM_FRO_SCALED, NORM_LITERAL = 0, 1

PART = dict(DEPTH=0, PERM=1, NODES=2, BOXES=3, NEAR_PTR=4, NEAR_IDX=5, FAR_PTR=6, FAR_IDX=7, RANKS=8,
            SKEL=9, BASIS=10, COUPLING=11, DENSE=12, TOP=13, SKEL_POS=14, RANKS_C=15, SKEL_C=16, BASIS_C=17,
            SKEL_POS_C=18)
PART_DTYPE = dict(DEPTH="i4", PERM="i4", NODES="i4", BOXES="f8", NEAR_PTR="i4", NEAR_IDX="i4", FAR_PTR="i4",
                  FAR_IDX="i4", RANKS="i4", SKEL="i4", BASIS="f8", COUPLING="f8", DENSE="f8", TOP="i4",
                  SKEL_POS="i4", RANKS_C="i4", SKEL_C="i4", BASIS_C="f8", SKEL_POS_C="i4")


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("leaf_size", C.c_int32), ("eta", C.c_double), ("d0", C.c_int32),
                ("d_inc", C.c_int32), ("d_max", C.c_int32), ("seed", C.c_uint64), ("precision", C.c_int32),
                ("norm_mode", C.c_int32), ("sketch_ahead", C.c_int32), ("oversample", C.c_int32)]


class Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("length", C.c_double), ("wavenumber", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("depth", C.c_int32), ("top", C.c_int32),
                ("samples", C.c_int32), ("sketched", C.c_int32), ("rounds", C.c_int32), ("rank_min", C.c_int32),
                ("rank_max", C.c_int32),
                ("delta", C.c_double), ("norm_estimate", C.c_double), ("near_blocks", C.c_int64),
                ("far_blocks", C.c_int64), ("bytes_dense", C.c_int64), ("bytes_coupling", C.c_int64),
                ("bytes_basis", C.c_int64), ("t_total", C.c_double), ("t_tree", C.c_double),
                ("t_sample", C.c_double), ("t_near_gen", C.c_double), ("t_subtract", C.c_double),
                ("t_convtest", C.c_double), ("t_id", C.c_double), ("t_upsweep", C.c_double),
                ("t_coupling", C.c_double), ("t_misc", C.c_double), ("t_host_plan", C.c_double),
                ("sketch_flops", C.c_double),
                ("sketch_entries", C.c_double), ("sketch_calls", C.c_int32), ("fixed_samples", C.c_int32),
                ("bytes_peak", C.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("points", C.c_void_p), ("kernel", Kernel),
                ("tol", C.c_double), ("leaf_size", C.c_int32), ("eta", C.c_double), ("d0", C.c_int32),
                ("d_inc", C.c_int32), ("seed", C.c_uint64), ("norm_mode", C.c_int32), ("oversample", C.c_int32)]


class BatchOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("d_max", C.c_int32), ("use_graph", C.c_int32),
                ("first_pass", C.c_int32), ("sketch_cols", C.c_int32), ("bsr_cols", C.c_int32)]


class BatchInfo(C.Structure):
    _fields_ = [("t_total_ms", C.c_double), ("t_plan_ms", C.c_double), ("t_setup_ms", C.c_double),
                ("t_capture_ms", C.c_double), ("t_device_ms", C.c_double), ("levels", C.c_int32),
                ("graph_nodes", C.c_int32), ("device_bytes", C.c_int64), ("sketch_flops", C.c_double),
                ("t_layout_ms", C.c_double), ("t_alloc_ms", C.c_double), ("t_results_ms", C.c_double),
                ("first_pass", C.c_int32), ("second_pass", C.c_int32), ("sketch_cols", C.c_int32),
                ("bsr_cols", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = C.c_void_p
# h2_sketch_fn(user, n, d, omega, ldo, y, ldy, stream)
SKETCH_FN = C.CFUNCTYPE(C.c_int, _P, C.c_int64, C.c_int32, _P, C.c_int64, _P, C.c_int64, _P)
# h2_entry_fn(user, nblocks, idx, rbeg, rcnt, cbeg, ccnt, off, out, max_rows, max_cols, stream)
ENTRY_FN = C.CFUNCTYPE(C.c_int, _P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, C.c_int32, C.c_int32, _P)
_SIGS = {
    "h2_opts_default": [C.POINTER(Opts)],
    "h2_status_string": [C.c_int],
    "h2_last_error": [],
    "h2_ctx_create": [C.c_int, _P, C.POINTER(_P)],
    "h2_ctx_destroy": [_P],
    "h2_plan_create": [C.c_int64, C.c_int32, _P, C.c_int32, C.c_double, C.POINTER(_P)],
    "h2_plan_create_device": [_P, C.c_int64, C.c_int32, _P, C.c_int32, C.c_double, C.POINTER(_P)],
    "h2_plan_free": [_P],
    "h2_plan_export": [_P, C.c_int32, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_size_t)],
    "h2_gaussian": [_P, C.c_uint64, C.c_int64, _P, C.c_int64, C.c_int32, _P, C.c_int64],
    "h2_sketch": [_P, C.c_int64, C.c_int32, _P, C.POINTER(Kernel), C.c_int32, C.c_int32, _P, C.c_int64, _P,
                  C.c_int64],
    "h2_build": [_P, C.c_int64, C.c_int32, _P, C.POINTER(Kernel), SKETCH_FN, _P, ENTRY_FN, _P, C.POINTER(Opts),
                 C.POINTER(_P)],
    "h2_matvec": [_P, _P, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.c_int64],
    "h2_matvec_noalloc": [_P, _P, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.c_int64],
    "h2_entries": [_P, _P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, C.c_int32, C.c_int32],
    "h2_export": [_P, C.c_int32, C.c_int32, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_size_t)],
    "h2_query": [_P, C.POINTER(Info)],
    "h2_free": [_P],
    "h2_build_batched": [_P, C.c_int32, C.POINTER(Problem), C.POINTER(BatchOpts), C.POINTER(_P),
                         C.POINTER(BatchInfo)],
    "h2_build_update": [_P, _P, C.c_int32, _P, C.c_int64, _P, C.c_int64, C.POINTER(Opts), C.POINTER(_P)],
    "h2_autotune_leaf": [_P, C.c_int32, C.POINTER(Problem), C.POINTER(BatchOpts), C.POINTER(C.c_int32), C.c_int32,
                         C.POINTER(C.c_int32)],
    "h2_autotune_tiles": [_P, C.c_int32, C.POINTER(Problem), C.POINTER(BatchOpts), C.POINTER(BatchOpts),
                          C.POINTER(C.c_double)],
}
EXPORTED = tuple(_SIGS)

_lib = None


class H2Error(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libh2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_16759_amd.build_lib`")
        lib = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = C.c_char_p if name in ("h2_status_string", "h2_last_error") else C.c_int
        _lib = lib
    return _lib


def check(status: int, func: str):
    if status != H2_OK:
        raise H2Error(status, func, load().h2_last_error().decode())
