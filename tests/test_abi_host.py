"""Host-side checks of libhepk.so that need no GPU.

The library loads, exports every function include/hepk.h declares, and
rejects invalid arguments with HEPK_EINVAL / HEPK_EUNSUPPORTED and a message
before anything is enqueued (no device call is made on these paths).
"""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1906_06242_amd import hepk as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hepk.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(H.LIB_PATH):
        from paper_1906_06242_amd import build
        build.build(verbose=False)
    return H.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hepk_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    for fn in ("hepk_select", "hepk_reduce", "hepk_match_dr", "hepk_hist_fill", "hepk_pipeline"):
        assert fn in names
    assert set(names) == set(H.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", H.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (hepk_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert getattr(lib, n) is not None


def test_abi_version(lib):
    v = int(re.search(r"#define HEPK_ABI_VERSION (\d+)", open(HEADER).read()).group(1))
    assert lib.hepk_abi_version() == v


def _rc(name, *args):
    return getattr(H.load(), name)(*args)


def test_select_rejects_bad_arguments(lib):
    cuts = (H.Cut * 9)()
    assert _rc("hepk_select", cuts, 9, 10, None, 1, None) == H.EINVAL
    assert "n_cuts" in H.last_error()
    assert _rc("hepk_select", cuts, 1, -1, None, 1, None) == H.EINVAL
    cuts[0] = H.Cut(8, 7, H.GT, 0.0, 0)
    assert _rc("hepk_select", cuts, 1, 10, None, 16, None) == H.EINVAL
    assert "dtype" in H.last_error()
    cuts[0] = H.Cut(8, H.F32, 17, 0.0, 0)
    assert _rc("hepk_select", cuts, 1, 10, None, 16, None) == H.EINVAL
    assert _rc("hepk_select", cuts, 0, 10, None, None, None) == H.EINVAL
    # nothing to do is not an error
    assert _rc("hepk_select", None, 0, 0, None, None, None) == H.OK


def test_reduce_rejects_bad_arguments(lib):
    assert _rc("hepk_reduce", 9, 8, 1, None, H.F32, None, None, 8, None, None, None) == H.EINVAL
    assert _rc("hepk_reduce", H.COUNT, None, 1, None, H.F32, None, None, 8, None, None, None) == H.EINVAL
    assert _rc("hepk_reduce", H.SUM, 8, 1, 8, H.I32, None, None, 8, None, None, None) == H.EUNSUPPORTED
    assert _rc("hepk_reduce", H.SUM, 8, 1, 8, H.F32, None, None, 8, None, 8, None) == H.EINVAL
    assert "COUNT" in H.last_error()
    assert _rc("hepk_reduce", H.SUM, 8, 1, 8, H.F32, None, None, 8, 8, None, None) == H.EINVAL
    assert _rc("hepk_reduce", H.COUNT, 8, -2, None, H.F32, None, None, 8, None, None, None) == H.EINVAL


def test_match_dr_rejects_bad_arguments(lib):
    a = [8, 8, 8, None, 8, 8, 8, None]
    assert _rc("hepk_match_dr", *a, H.I32, 5, C.c_float(0.4), 8, None, None, None) == H.EUNSUPPORTED
    assert _rc("hepk_match_dr", *a, H.F32, -1, C.c_float(0.4), 8, None, None, None) == H.EINVAL
    b = list(a)
    b[0] = None
    assert _rc("hepk_match_dr", *b, H.F32, 5, C.c_float(0.4), 8, None, None, None) == H.EINVAL


def test_hist_fill_rejects_bad_arguments(lib):
    h = H.Hist(8, 0, 8, 8)
    assert _rc("hepk_hist_fill", 8, H.F32, None, None, 10, C.byref(h), None) == H.EINVAL
    assert "nbins" in H.last_error()
    h = H.Hist(8, 10, None, 8)
    assert _rc("hepk_hist_fill", 8, H.F32, None, None, 10, C.byref(h), None) == H.EINVAL
    h = H.Hist(8, 10, 8, 8)
    assert _rc("hepk_hist_fill", 8, 5, None, None, 10, C.byref(h), None) == H.EINVAL
    assert _rc("hepk_hist_fill", 8, H.F32, None, None, 10, None, None) == H.EINVAL


def test_plan_create_rejects_bad_arguments(lib):
    out = C.c_void_p()
    ds = (H.DatasetS * 1)()
    q = (H.QueryS * 1)()
    assert _rc("hepk_plan_create", ds, 0, q, 1, None, C.byref(out)) == H.EINVAL
    ds[0].dtype = H.I32
    assert _rc("hepk_plan_create", ds, 1, q, 1, None, C.byref(out)) == H.EINVAL
    ds[0].dtype = H.F32
    ds[0].n_events = 10
    assert _rc("hepk_plan_create", ds, 1, q, 1, None, C.byref(out)) == H.EINVAL
    assert "offsets" in H.last_error()
    ds[0].jets = H.Collection(8, 8, 8, 8, None)
    ds[0].muons = H.Collection(8, 8, 8, 8, 8)
    q[0].n_scale = 0
    assert _rc("hepk_plan_create", ds, 1, q, 1, None, C.byref(out)) == H.EINVAL
    assert "scale" in H.last_error()
    sc = (C.c_float * 1)(1.0)
    q[0].n_scale = 1
    q[0].scales = C.cast(sc, C.c_void_p)
    assert _rc("hepk_plan_create", ds, 1, q, 1, None, C.byref(out)) == H.EINVAL  # nbins 0
    edges = (C.c_float * 11)(*range(11))
    for h in range(3):
        q[0].edges[h] = C.cast(edges, C.c_void_p)
        q[0].nbins[h] = 10
    bad = H.Tune(384, 1, 0, 0)
    assert _rc("hepk_plan_create", ds, 1, q, 1, C.byref(bad), C.byref(out)) == H.EINVAL
    assert "block" in H.last_error()
    bad = H.Tune(256, 3, 0, 0)
    assert _rc("hepk_plan_create", ds, 1, q, 1, C.byref(bad), C.byref(out)) == H.EINVAL
    bad = H.Tune(1024, 2, 0, 0)
    assert _rc("hepk_plan_create", ds, 1, q, 1, C.byref(bad), C.byref(out)) == H.EINVAL
    assert "1024" in H.last_error()
    ds[0].n_events = 1 << 31
    assert _rc("hepk_plan_create", ds, 1, q, 1, None, C.byref(out)) == H.EINVAL
    assert not out.value


def test_stream_read_rejects_bad_arguments(lib):
    assert _rc("hepk_stream_read", None, 16, 8, None) == H.EINVAL
    assert _rc("hepk_stream_read", 16, 15, 8, None) == H.EINVAL
    assert "multiple of 16" in H.last_error()
    assert _rc("hepk_stream_read", 8, 16, 8, None) == H.EINVAL
    assert "aligned" in H.last_error()
    assert _rc("hepk_stream_read", 16, 0, 8, None) == H.OK


def test_pipeline_and_queries_reject_null(lib):
    assert _rc("hepk_pipeline", None, 8, 8, None) == H.EINVAL
    n = C.c_int64()
    assert _rc("hepk_plan_hist_slots", None, C.byref(n)) == H.EINVAL
    assert _rc("hepk_plan_destroy", None) == H.OK
    assert _rc("hepk_validate_offsets", None, 1, 1, 8, None) == H.EINVAL


def test_slot_range_graph_autotune_reject_bad_arguments(lib):
    assert _rc("hepk_plan_set_query", None, 0, None, None) == H.EINVAL
    assert _rc("hepk_pipeline_range", None, 0, 1, 8, 8, None) == H.EINVAL
    assert _rc("hepk_pipeline_graph", None, 8, 8, None) == H.EINVAL
    best = H.Tune()
    ds = (H.DatasetS * 1)()
    q = (H.QueryS * 1)()
    assert _rc("hepk_autotune", ds, 1, q, 1, 8, 8, 0, C.byref(best), None, None) == H.EINVAL
    assert "reps" in H.last_error()
    assert _rc("hepk_autotune", ds, 1, q, 1, None, 8, 3, C.byref(best), None, None) == H.EINVAL
    out = C.c_void_p()
    opts = H.PlanOpts(H.Tune(0, 0, 0, 0), 0, -5)
    ds[0] = H.DatasetS(0, H.F32, H.Collection(8, 8, 8, 8, None), H.Collection(8, 8, 8, 8, 8),
                       H.Collection(None, None, None, None, None), None)
    sc = (C.c_float * 1)(1.0)
    e = (C.c_float * 3)(0.0, 1.0, 2.0)
    q[0].n_scale = 1
    q[0].scales = C.cast(sc, C.c_void_p)
    for h in range(3):
        q[0].edges[h] = C.cast(e, C.c_void_p)
        q[0].nbins[h] = 2
    assert _rc("hepk_plan_create_ex", ds, 1, q, 1, C.byref(opts), C.byref(out)) == H.EINVAL
    assert "reserve_bins" in H.last_error()
    for v in (0.0, -1.0, float("inf"), float("nan")):
        sc[0] = v
        assert _rc("hepk_plan_create_ex", ds, 1, q, 1, C.byref(opts), C.byref(out)) == H.EINVAL
        assert "positive" in H.last_error()
    sc[0] = 1.0
    bad = (C.c_float * 3)(0.0, 2.0, 1.0)
    q[0].edges[1] = C.cast(bad, C.c_void_p)
    opts = H.PlanOpts(H.Tune(0, 0, 0, 0), 0, 0)
    assert _rc("hepk_plan_create_ex", ds, 1, q, 1, C.byref(opts), C.byref(out)) == H.EINVAL
    assert "increasing" in H.last_error()


def test_autotune_cache_hit_needs_no_device(tmp_path):
    """A stored launch-configuration search result is returned for the same
    device and workload without searching (no device call on this path)."""
    import json
    from paper_1906_06242_amd import datagen

    class Fake:  # the fields workload_key reads of a resident dataset
        def __init__(self, n):
            self.n_events, self.content_dtype = n, "f32"
            self.tensors = {"jets.offsets": None, "muons.offsets": None}
    dds, qs = [Fake(1000), Fake(20)], [datagen.Query()]
    key = H.workload_key(dds, qs, device="dev0")
    assert key != H.workload_key([Fake(1001), Fake(20)], qs, device="dev0")
    assert key != H.workload_key(dds, qs, device="dev1")
    assert key != H.workload_key(dds, [datagen.Query(scales=datagen.jes_scales())], device="dev0")
    path = tmp_path / "autotune.json"
    path.write_text(json.dumps({key: {"tune": {"block": 256, "ev_per_thread": 2, "hist_mode": 0, "grid": 0},
                                      "ms": 1.5}}))
    best, ms = H.autotune(dds, qs, cache=str(path), device="dev0")
    assert best["block"] == 256 and best["ev_per_thread"] == 2 and ms == 1.5
