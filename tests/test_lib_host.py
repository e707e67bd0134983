"""CPU checks of libh2: it loads, exports every declared symbol, and its host
cluster plan (tree + interaction lists) equals the oracle's bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2506_16759_amd as h2
from paper_2506_16759_amd import _lib
from paper_2506_16759_amd.workloads import CUBE_131K, SMALL_2D, batch_problems, uniform_points
from oracle.tree import build_lists, build_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "h2.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(h2_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTED)


def test_precision_constants_match_the_header():
    text = open(os.path.join(ROOT, "include", "h2.h")).read()
    body = re.search(r"typedef enum \{([^}]*)\} h2_precision;", text).group(1)
    values = {k: int(v) for k, v in re.findall(r"H2_(\w+)\s*=\s*(\d+)", body)}
    assert values == {"FP64": h2.FP64, "FP32": h2.FP32, "BF16X3": h2.BF16X3, "FP32E": h2.FP32E,
                      "BF16X6": h2.BF16X6, "FP64_SYM": h2.FP64_SYM}


def test_status_strings_and_defaults():
    lib = _lib.load()
    assert lib.h2_status_string(-5).decode() == "adaptive sampling reached d_max"
    o = h2.opts_default()
    assert (o.tol, o.leaf_size, o.eta, o.d0, o.d_inc, o.d_max) == (1e-6, 64, 0.7, 32, 16, 256)
    assert (o.sketch_ahead, o.oversample) == (32, 0)


def _compare_plan(pts, leaf, eta):
    p = h2.plan_create(pts, leaf, eta)
    tr = build_tree(pts, leaf)
    L = build_lists(tr, eta)
    D = int(p.export("DEPTH")[0])
    assert D == tr.depth
    np.testing.assert_array_equal(p.export("PERM"), tr.perm)
    nodes = p.export("NODES").reshape(-1, 2)
    np.testing.assert_array_equal(nodes[:, 0], tr.begin)
    np.testing.assert_array_equal(nodes[:, 1], tr.end)
    boxes = p.export("BOXES").reshape(-1, 2, pts.shape[0])
    np.testing.assert_array_equal(boxes[:, 0], tr.lo)
    np.testing.assert_array_equal(boxes[:, 1], tr.hi)
    np.testing.assert_array_equal(p.export("NEAR_PTR"), L.near_ptr)
    np.testing.assert_array_equal(p.export("NEAR_IDX"), L.near_idx)
    for t in range(D + 1):
        np.testing.assert_array_equal(p.export("FAR_PTR", t), L.far_ptr[t])
        np.testing.assert_array_equal(p.export("FAR_IDX", t), L.far_idx[t])
    return p, tr, L


@pytest.mark.parametrize("n,dim,leaf,eta,seed", [
    (4096, 2, 64, 0.7, 0), (5000, 3, 64, 0.7, 3), (777, 3, 20, 0.5, 1), (1000, 1, 8, 1.0, 2),
    (33, 2, 2, 0.7, 5), (50, 3, 64, 0.7, 6), (3000, 2, 37, 2.0, 7),
])
def test_plan_bit_exact_with_oracle(n, dim, leaf, eta, seed):
    _compare_plan(uniform_points(n, dim, seed), leaf, eta)


def test_plan_bit_exact_small_2d_workload():
    w = SMALL_2D
    _compare_plan(w.points(), w.leaf_size, w.eta)


@pytest.mark.slow
def test_plan_bit_exact_full_cube_workload():
    w = CUBE_131K
    _compare_plan(w.points(), w.leaf_size, w.eta)


def test_plan_bit_exact_batch_sizes():
    # ragged sizes and both dimensions of the batched workload (first few problems)
    for w in batch_problems()[:4]:
        _compare_plan(w.points(), w.leaf_size, w.eta)


def test_plan_duplicates_and_grid_ties():
    pts = np.repeat(uniform_points(200, 2, 9), 3, axis=1)
    _compare_plan(pts, 8, 0.7)
    g = np.stack(np.meshgrid(np.arange(16.0), np.arange(16.0)), 0).reshape(2, -1)   # exact ties everywhere
    _compare_plan(np.ascontiguousarray(g), 4, 0.7)


@pytest.mark.parametrize("kwargs,msg", [
    (dict(leaf=1), "leaf_size"), (dict(eta=0.0), "eta"), (dict(eta=float("nan")), "eta"),
    (dict(nan=True), "finite"), (dict(dim=4), "dim"),
])
def test_plan_rejects_bad_arguments(kwargs, msg):
    dim = kwargs.get("dim", 2)
    pts = np.random.default_rng(0).random((dim, 100))
    if kwargs.get("nan"):
        pts[0, 5] = np.nan
    with pytest.raises(h2.H2Error) as ei:
        h2.plan_create(pts, kwargs.get("leaf", 8), kwargs.get("eta", 0.7))
    assert ei.value.status == -1 and msg in str(ei.value)


def test_export_size_query_and_small_buffer():
    p = h2.plan_create(uniform_points(500, 2, 0), 16, 0.7)
    lib = _lib.load()
    need = ctypes.c_size_t(0)
    assert lib.h2_plan_export(p._h, _lib.PART["PERM"], 0, None, 0, ctypes.byref(need)) == 0
    assert need.value == 500 * 4
    buf = (ctypes.c_int32 * 10)()
    assert lib.h2_plan_export(p._h, _lib.PART["PERM"], 0, buf, 40, ctypes.byref(need)) == -1
    assert lib.h2_plan_export(p._h, _lib.PART["FAR_PTR"], 99, None, 0, ctypes.byref(need)) == -1


def test_batched_build_rejects_bad_arguments_before_any_device_work():
    import ctypes as C

    from paper_2506_16759_amd import _lib
    lib = _lib.load()
    handles = (C.c_void_p * 1)()
    bo = _lib.BatchOpts(0, 64, 1)
    prob = (_lib.Problem * 1)()
    # NULL context
    assert lib.h2_build_batched(None, 1, prob, C.byref(bo), handles, None) == -1
    assert "NULL" in lib.h2_last_error().decode()
    assert handles[0] is None


def test_autotune_rejects_bad_arguments_before_any_device_work():
    import ctypes as C

    from paper_2506_16759_amd import _lib
    lib = _lib.load()
    prob = (_lib.Problem * 1)()
    bo = _lib.BatchOpts(0, 64, 1)
    cand = (C.c_int32 * 1)(64)
    best = (C.c_int32 * 1)()
    assert lib.h2_autotune_leaf(None, 1, prob, C.byref(bo), cand, 1, best) == -1


def test_tile_autotune_rejects_bad_arguments_before_any_device_work():
    import ctypes as C

    from paper_2506_16759_amd import _lib
    lib = _lib.load()
    prob = (_lib.Problem * 1)()
    bo = _lib.BatchOpts(0, 64, 1)
    tuned = _lib.BatchOpts()
    assert lib.h2_autotune_tiles(None, 1, prob, C.byref(bo), C.byref(tuned), None) == -1
    assert "NULL" in lib.h2_last_error().decode()


def test_device_plan_rejects_null_context():
    import ctypes as C

    from paper_2506_16759_amd import _lib
    lib = _lib.load()
    out = C.c_void_p()
    assert lib.h2_plan_create_device(None, 100, 3, None, 64, 0.7, C.byref(out)) == -1
    assert "NULL" in lib.h2_last_error().decode()
    assert out.value is None


def test_traffic_summary_scales_by_the_copy(tmp_path):
    """bench.py --traffic-from: KiB counters scaled so that the 1 GiB copy reads
    and writes exactly 1 GiB; the first launch of each sketch variant counts."""
    import bench
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    sk = "void h2dev::(anonymous namespace)::sketch_f64_kernel<3, 1, 64>(long, double const*)"
    for counter, copy_kib, sk_kib in (("FETCH_SIZE", 2 ** 19, 1000.0), ("WRITE_SIZE", 2 ** 20, 64.0)):
        d = tmp_path / counter
        d.mkdir()
        (d / "run_counter_collection.csv").write_text(
            hdr + f'1,"{sk}",{counter},{sk_kib / 2}\n1,"{sk}",{counter},{sk_kib / 2}\n'
            f'2,"{sk}",{counter},{9 * sk_kib}\n3,"__amd_rocclr_copyBuffer",{counter},{copy_kib}\n')
    rec = bench.traffic_summary(str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE"))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    k = rec["kernels"]["sketch_f64_kernel<3,exp,64>"]
    assert k["fetch_bytes"] == 1000.0 * 2.0 * 1024 and k["write_bytes"] == 64.0 * 1024
    assert rec["source_sha256"] == bench.sketch_source_digest()
