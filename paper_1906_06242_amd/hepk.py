"""Python binding of libhepk.so (include/hepk.h): argument marshalling only.

Every function takes torch tensors that live on the current HIP device,
passes their device pointers and the current stream to the C ABI, and
raises HepkError on a non-OK status.  Every step of the analysis runs in the
library's HIP kernels; there is no host fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhepk.so")

OK, EINVAL, EHIP, EUNSUPPORTED, ENOMEM = 0, -1, -2, -3, -4
F32, F16, I32, U8 = 0, 1, 2, 3
GT, GE, LT, LE, ABS_LT, ABS_LE = range(6)
COUNT, SUM, MAX, MIN, ARGMAX, ARGMIN, PROD = range(7)
MAX_CUTS = 8

EXPORTS = (
    "hepk_select", "hepk_reduce", "hepk_match_dr", "hepk_hist_fill", "hepk_validate_offsets", "hepk_stream_read",
    "hepk_plan_create", "hepk_plan_create_ex", "hepk_plan_set_query", "hepk_plan_hist_slots",
    "hepk_plan_hist_offset", "hepk_plan_get_tune", "hepk_pipeline", "hepk_pipeline_range",
    "hepk_pipeline_graph", "hepk_autotune", "hepk_plan_destroy", "hepk_last_error", "hepk_abi_version",
    "hepk_plan_debug_layout", "hepk_pipeline_debug",
    "hepk_hist_fill_w2", "hepk_get_bin_contents", "hepk_interp", "hepk_jes_delta",
    "hepk_pipeline_noalloc", "hepk_pipeline_w2",
    "hepk_get_in_offsets", "hepk_set_in_offsets", "hepk_select_opposite_sign", "hepk_compact",
    "hepk_p4", "hepk_best_triplet",
    "hepk_streamer_create", "hepk_streamer_hist_slots", "hepk_stream_pass", "hepk_streamer_destroy",
    "hepk_plan_set_query_at",
)

# hepk_event_record, as a numpy structured dtype (32 bytes)
EVENT_RECORD = [("n_mu", "<i4"), ("n_jet", "<i4"), ("n_b", "<i4"), ("state", "<i4"),
                ("ht", "<f4"), ("lead", "<f4"), ("w", "<f4"), ("reserved", "<i4")]
REC_SKIPPED, REC_FAILS, REC_PASSES = 1, 2, 3


class HepkError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


class Cut(C.Structure):
    _fields_ = [("col", C.c_void_p), ("dtype", C.c_int32), ("op", C.c_int32),
                ("thr", C.c_float), ("ithr", C.c_int32)]


class Hist(C.Structure):
    _fields_ = [("edges", C.c_void_p), ("nbins", C.c_int32),
                ("sumw", C.c_void_p), ("counts", C.c_void_p)]


class Collection(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("pt", C.c_void_p), ("eta", C.c_void_p),
                ("phi", C.c_void_p), ("extra", C.c_void_p)]


class DatasetS(C.Structure):
    _fields_ = [("n_events", C.c_int64), ("dtype", C.c_int32),
                ("jets", Collection), ("muons", Collection), ("electrons", Collection),
                ("weights", C.c_void_p), ("npu", C.c_void_p)]


class QueryS(C.Structure):
    _fields_ = [("mu_pt", C.c_float), ("mu_abseta", C.c_float), ("mu_iso", C.c_float),
                ("el_pt", C.c_float), ("el_abseta", C.c_float),
                ("jet_pt", C.c_float), ("jet_abseta", C.c_float),
                ("dr", C.c_float), ("btag", C.c_float),
                ("min_mu", C.c_int32), ("min_jet", C.c_int32), ("min_b", C.c_int32),
                ("n_scale", C.c_int32), ("scales", C.c_void_p),
                ("edges", C.c_void_p * 3), ("nbins", C.c_int32 * 3),
                ("pu_edges", C.c_void_p), ("pu_contents", C.c_void_p), ("pu_nbins", C.c_int32),
                ("sf_edges", C.c_void_p), ("sf_contents", C.c_void_p), ("sf_nbins", C.c_int32),
                ("jes_mode", C.c_int32), ("jes_eta_edges", C.c_void_p), ("jes_pt_edges", C.c_void_p),
                ("jes_delta", C.c_void_p), ("jes_n_eta", C.c_int32), ("jes_n_pt", C.c_int32)]


class Tune(C.Structure):
    _fields_ = [("block", C.c_int32), ("ev_per_thread", C.c_int32),
                ("hist_mode", C.c_int32), ("grid", C.c_int32)]

    def as_dict(self):
        return {"block": self.block, "ev_per_thread": self.ev_per_thread,
                "hist_mode": self.hist_mode, "grid": self.grid}

    @classmethod
    def of(cls, d: Optional[dict]) -> "Tune":
        d = d or {}
        return cls(d.get("block", 512), d.get("ev_per_thread", 1), d.get("hist_mode", 0), d.get("grid", 0))


class StreamOpts(C.Structure):
    _fields_ = [("batch_events", C.c_int64), ("n_buffers", C.c_int32), ("host_threads", C.c_int32),
                ("tune", Tune)]


class PlanOpts(C.Structure):
    _fields_ = [("tune", Tune), ("shared_hist", C.c_int32), ("reserve_bins", C.c_int32), ("sumw2", C.c_int32),
                ("hist_arena_slots", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libhepk.so (built in-tree by paper_1906_06242_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() "
                           "(or python paper_1906_06242_amd/build.py) first")
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.hepk_select.argtypes = [C.POINTER(Cut), i32, i64, vp, vp, vp]
    lib.hepk_reduce.argtypes = [i32, vp, i64, vp, i32, vp, vp, vp, vp, vp, vp]
    lib.hepk_match_dr.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i32, i64, C.c_float, vp, vp, vp, vp]
    lib.hepk_hist_fill.argtypes = [vp, i32, vp, vp, i64, C.POINTER(Hist), vp]
    lib.hepk_hist_fill_w2.argtypes = [vp, i32, vp, vp, i64, C.POINTER(Hist), vp, vp]
    lib.hepk_get_bin_contents.argtypes = [vp, i32, i64, vp, i32, vp, vp, vp]
    lib.hepk_interp.argtypes = [vp, i32, i64, vp, i32, vp, vp, vp]
    lib.hepk_jes_delta.argtypes = [vp, vp, i32, i64, vp, i32, vp, i32, vp, vp, vp]
    lib.hepk_get_in_offsets.argtypes = [vp, i64, vp, i32, vp, vp, vp, i32, C.c_float, vp, vp, vp]
    lib.hepk_set_in_offsets.argtypes = [vp, i64, vp, i32, vp, vp, vp, i32, C.c_float, vp]
    lib.hepk_select_opposite_sign.argtypes = [vp, i64, vp, i32, vp, vp, vp, vp]
    lib.hepk_compact.argtypes = [vp, i64, vp, i32, vp, vp, i64, vp, vp]
    lib.hepk_p4.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp]
    lib.hepk_best_triplet.argtypes = [vp, i64, vp, vp, vp, vp, vp, C.c_float, vp, vp, vp]
    lib.hepk_streamer_create.argtypes = [C.POINTER(DatasetS), C.POINTER(QueryS), i32, C.POINTER(StreamOpts),
                                         C.POINTER(vp)]
    lib.hepk_streamer_hist_slots.argtypes = [vp, C.POINTER(i64)]
    lib.hepk_stream_pass.argtypes = [vp, vp, vp, vp]
    lib.hepk_streamer_destroy.argtypes = [vp]
    lib.hepk_validate_offsets.argtypes = [vp, i64, i64, vp, vp]
    lib.hepk_stream_read.argtypes = [vp, i64, vp, vp]
    lib.hepk_plan_create.argtypes = [C.POINTER(DatasetS), i32, C.POINTER(QueryS), i32,
                                     C.POINTER(Tune), C.POINTER(vp)]
    lib.hepk_plan_create_ex.argtypes = [C.POINTER(DatasetS), i32, C.POINTER(QueryS), i32,
                                        C.POINTER(PlanOpts), C.POINTER(vp)]
    lib.hepk_plan_set_query.argtypes = [vp, i32, C.POINTER(QueryS), vp]
    lib.hepk_plan_set_query_at.argtypes = [vp, i32, C.POINTER(QueryS), i64, vp]
    lib.hepk_pipeline_range.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.hepk_pipeline_graph.argtypes = [vp, vp, vp, vp]
    lib.hepk_autotune.argtypes = [C.POINTER(DatasetS), i32, C.POINTER(QueryS), i32, vp, vp, i32,
                                  C.POINTER(Tune), C.POINTER(C.c_float), vp]
    lib.hepk_plan_hist_slots.argtypes = [vp, C.POINTER(i64)]
    lib.hepk_plan_hist_offset.argtypes = [vp, i32, i32, i32, i32, C.POINTER(i64), C.POINTER(i32)]
    lib.hepk_plan_get_tune.argtypes = [vp, C.POINTER(Tune)]
    lib.hepk_pipeline.argtypes = [vp, vp, vp, vp]
    lib.hepk_pipeline_w2.argtypes = [vp, vp, vp, vp, vp]
    lib.hepk_plan_debug_layout.argtypes = [vp, i32, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    lib.hepk_pipeline_debug.argtypes = [vp, vp, vp, vp, vp]
    lib.hepk_plan_destroy.argtypes = [vp]
    lib.hepk_pipeline_noalloc.argtypes = [C.POINTER(DatasetS), i32, C.POINTER(QueryS), i32, C.POINTER(Tune),
                                          vp, vp, vp]
    lib.hepk_last_error.restype = C.c_char_p
    lib.hepk_last_error.argtypes = []
    lib.hepk_abi_version.restype = C.c_int
    for name in EXPORTS:
        if name not in ("hepk_last_error", "hepk_abi_version"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().hepk_last_error().decode()


def _call(name: str, *args) -> None:
    rc = getattr(load(), name)(*args)
    if rc != OK:
        raise HepkError(name, rc, last_error())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("hepk expects device tensors")
    if not t.is_contiguous():
        raise ValueError("hepk expects contiguous tensors")
    return t.data_ptr()


def _stream(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def dtype_code(t) -> int:
    import torch
    return {torch.float32: F32, torch.float16: F16, torch.int32: I32, torch.uint8: U8}[t.dtype]


# ---------------------------------------------------------------- primitives

def select(cuts: Sequence, n: int, mask_in=None, out=None, stream=None):
    """cuts: [(column tensor, op, threshold)]; returns a uint8 mask of n rows."""
    import torch
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device="cuda")
    arr = (Cut * max(1, len(cuts)))()
    for i, (col, op, thr) in enumerate(cuts):
        dt = dtype_code(col)
        if dt == I32:
            arr[i] = Cut(_ptr(col), dt, op, 0.0, int(thr))
        else:
            arr[i] = Cut(_ptr(col), dt, op, float(thr), 0)
    _call("hepk_select", arr, len(cuts), n, _ptr(mask_in), _ptr(out), _stream(stream))
    return out


def reduce(op: int, offsets, content=None, obj_mask=None, evt_mask=None, want_arg=False,
           want_offsets=False, out=None, stream=None):
    import torch
    n = offsets.numel() - 1
    if out is None:
        dt = torch.int32 if op in (COUNT, ARGMAX, ARGMIN) else torch.float32
        out = torch.empty(n, dtype=dt, device="cuda")
    arg = torch.empty(n, dtype=torch.int32, device="cuda") if want_arg else None
    offo = torch.empty(n + 1, dtype=torch.int64, device="cuda") if want_offsets else None
    dt = dtype_code(content) if content is not None else F32
    _call("hepk_reduce", op, _ptr(offsets), n, _ptr(content), dt, _ptr(obj_mask), _ptr(evt_mask),
          _ptr(out), _ptr(arg), _ptr(offo), _stream(stream))
    res = [out] + ([arg] if want_arg else []) + ([offo] if want_offsets else [])
    return res[0] if len(res) == 1 else tuple(res)


def match_dr(off_a, eta_a, phi_a, off_b, eta_b, phi_b, dr: float, mask_a=None, mask_b=None,
             want=("min_dr2", "idx", "clean"), stream=None):
    import torch
    ma = eta_a.numel()
    md = torch.empty(ma, dtype=torch.float32, device="cuda") if "min_dr2" in want else None
    ix = torch.empty(ma, dtype=torch.int32, device="cuda") if "idx" in want else None
    cl = torch.empty(ma, dtype=torch.uint8, device="cuda") if "clean" in want else None
    _call("hepk_match_dr", _ptr(off_a), _ptr(eta_a), _ptr(phi_a), _ptr(mask_a), _ptr(off_b),
          _ptr(eta_b), _ptr(phi_b), _ptr(mask_b), dtype_code(eta_a), off_a.numel() - 1, dr,
          _ptr(md), _ptr(ix), _ptr(cl), _stream(stream))
    return md, ix, cl


def hist_fill(x, edges, sumw, counts, w=None, evt_mask=None, sumw2=None, stream=None):
    """Accumulating weighted fill; with sumw2 also the squared weights (hepk_hist_fill_w2)."""
    h = Hist(_ptr(edges), edges.numel() - 1, _ptr(sumw), _ptr(counts))
    if sumw2 is None:
        _call("hepk_hist_fill", _ptr(x), dtype_code(x), _ptr(w), _ptr(evt_mask), x.numel(),
              C.byref(h), _stream(stream))
    else:
        _call("hepk_hist_fill_w2", _ptr(x), dtype_code(x), _ptr(w), _ptr(evt_mask), x.numel(),
              C.byref(h), _ptr(sumw2), _stream(stream))
    return sumw, counts


def _f32_out(n: int, out):
    import torch
    return torch.empty(n, dtype=torch.float32, device="cuda") if out is None else out


def get_bin_contents(x, edges, contents, out=None, stream=None):
    """Content of the lookup-histogram slot holding each element (contents: nbins+2)."""
    out = _f32_out(x.numel(), out)
    _call("hepk_get_bin_contents", _ptr(x), dtype_code(x), x.numel(), _ptr(edges), edges.numel() - 1,
          _ptr(contents), _ptr(out), _stream(stream))
    return out


def interp(x, edges, contents, out=None, stream=None):
    """Linear interpolation between the lookup histogram's bin centres."""
    out = _f32_out(x.numel(), out)
    _call("hepk_interp", _ptr(x), dtype_code(x), x.numel(), _ptr(edges), edges.numel() - 1,
          _ptr(contents), _ptr(out), _stream(stream))
    return out


def jes_delta(pt, eta, eta_edges, pt_edges, delta, out=None, stream=None):
    """Jet-energy-scale shift per object from the (|eta| row, pt) table delta[n_eta, n_pt]."""
    out = _f32_out(pt.numel(), out)
    _call("hepk_jes_delta", _ptr(pt), _ptr(eta), dtype_code(pt), pt.numel(), _ptr(eta_edges),
          eta_edges.numel() - 1, _ptr(pt_edges), pt_edges.numel() - 1, _ptr(delta), _ptr(out),
          _stream(stream))
    return out


def get_in_offsets(offsets, content, n: int = 0, idx=None, obj_mask=None, evt_mask=None, fill: float = 0.0,
                   stream=None):
    """(value float32[N], local index int32[N]) of the n-th selected object of every event."""
    import torch
    nev = offsets.numel() - 1
    out = torch.empty(nev, dtype=torch.float32, device="cuda")
    oi = torch.empty(nev, dtype=torch.int32, device="cuda")
    _call("hepk_get_in_offsets", _ptr(offsets), nev, _ptr(content), dtype_code(content), _ptr(obj_mask),
          _ptr(evt_mask), _ptr(idx), n, fill, _ptr(out), _ptr(oi), _stream(stream))
    return out, oi


def set_in_offsets(offsets, content, value: float, n: int = 0, idx=None, obj_mask=None, evt_mask=None,
                   stream=None):
    """Sets, in place, the n-th selected object of every event (content float32 or uint8)."""
    _call("hepk_set_in_offsets", _ptr(offsets), offsets.numel() - 1, _ptr(content), dtype_code(content),
          _ptr(obj_mask), _ptr(evt_mask), _ptr(idx), n, value, _stream(stream))
    return content


def select_opposite_sign(offsets, pt, charge, obj_mask=None, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty(pt.numel(), dtype=torch.uint8, device="cuda")
    _call("hepk_select_opposite_sign", _ptr(offsets), offsets.numel() - 1, _ptr(pt), dtype_code(pt),
          _ptr(charge), _ptr(obj_mask), _ptr(out), _stream(stream))
    return out


def compact(offsets, content, offsets_out, n_out: int, obj_mask=None, out=None, stream=None):
    """The selected objects of content, contiguous, laid out by offsets_out (n_out of them)."""
    import torch
    if out is None:
        out = torch.empty(max(1, n_out), dtype=content.dtype, device="cuda")
    _call("hepk_compact", _ptr(offsets), offsets.numel() - 1, _ptr(content), dtype_code(content), _ptr(obj_mask),
          _ptr(offsets_out), n_out, _ptr(out), _stream(stream))
    return out[:n_out]


def p4(pt, eta, phi, mass, stream=None):
    import torch
    o = [torch.empty(pt.numel(), dtype=torch.float32, device="cuda") for _ in range(4)]
    _call("hepk_p4", _ptr(pt), _ptr(eta), _ptr(phi), _ptr(mass), pt.numel(), *[_ptr(a) for a in o],
          _stream(stream))
    return tuple(o)


def best_triplet(offsets, px, py, pz, en, obj_mask=None, target: float = 172.0, stream=None):
    """(mass float32[N], local indices int32[N, 3]) of each event's triplet closest to target."""
    import torch
    nev = offsets.numel() - 1
    m = torch.empty(nev, dtype=torch.float32, device="cuda")
    ix = torch.empty(3 * max(nev, 0), dtype=torch.int32, device="cuda")
    _call("hepk_best_triplet", _ptr(offsets), nev, _ptr(px), _ptr(py), _ptr(pz), _ptr(en), _ptr(obj_mask),
          target, _ptr(m), _ptr(ix), _stream(stream))
    return m, ix.view(nev, 3)


def validate_offsets(offsets, n_objects: int, stream=None) -> int:
    import torch
    bad = torch.empty(1, dtype=torch.int64, device="cuda")
    _call("hepk_validate_offsets", _ptr(offsets), offsets.numel() - 1, n_objects, _ptr(bad),
          _stream(stream))
    return int(bad.item())


def stream_read(t, sink, stream=None):
    """Reads all of device tensor t (measurement helper; see hepk_stream_read)."""
    _call("hepk_stream_read", _ptr(t), t.numel() * t.element_size(), _ptr(sink), _stream(stream))


# ---------------------------------------------------------------- fused pass

class DeviceDataset:
    """Event columns resident in device memory.

    Built from a datagen.Dataset (host arrays are uploaded) or, with
    from_tensors, from device tensors keyed "jets.offsets", "jets.pt", ...,
    "weight".  view(e0, e1) is events [e0, e1) without copying: the offsets
    pointers move by e0 and still index the full content arrays.
    """

    def __init__(self, ds=None, device="cuda"):
        import numpy as np
        import torch
        self.tensors: Dict[str, "torch.Tensor"] = {}
        self.e0 = 0
        if ds is None:
            return
        self.n_events = ds.n_events
        self.content_dtype = ds.content_dtype
        for cname, coll in ds.collections():
            self.tensors[f"{cname}.offsets"] = torch.from_numpy(coll.offsets).to(device)
            for k, v in coll.cols.items():
                if k == "mass":
                    continue  # stored in the dataset, never read by the analysis
                if v.size == 0:  # keep a valid (never read) pointer for empty columns
                    v = np.zeros(1, v.dtype)
                self.tensors[f"{cname}.{k}"] = torch.from_numpy(v).to(device)
        w = ds.weight if ds.weight.size else np.ones(1, np.float32)
        self.tensors["weight"] = torch.from_numpy(w).to(device)
        if getattr(ds, "npu", None) is not None:
            npu = ds.npu if ds.npu.size else np.zeros(1, np.float32)
            self.tensors["npu"] = torch.from_numpy(np.ascontiguousarray(npu, np.float32)).to(device)

    @classmethod
    def from_tensors(cls, t: dict) -> "DeviceDataset":
        import torch
        d = cls()
        d.n_events = int(t["n_events"])
        d.content_dtype = t.get("content_dtype", "f32")
        for k, v in t.items():
            if isinstance(v, torch.Tensor):
                if v.numel() == 0:
                    v = torch.zeros(1, dtype=v.dtype, device=v.device)
                d.tensors[k] = v
        return d

    def view(self, e0: int, e1: int) -> "DeviceDataset":
        d = DeviceDataset()
        d.tensors = self.tensors
        d.content_dtype = self.content_dtype
        d.n_events = e1 - e0
        d.e0 = self.e0 + e0
        return d

    @property
    def has_electrons(self) -> bool:
        return "electrons.offsets" in self.tensors

    def t(self, key):
        return self.tensors.get(key)

    def struct(self) -> DatasetS:
        def coll(name, extra):
            off = self.t(f"{name}.offsets")
            if off is None:
                return Collection(None, None, None, None, None)
            return Collection(_ptr(off) + 8 * self.e0, _ptr(self.t(f"{name}.pt")),
                              _ptr(self.t(f"{name}.eta")), _ptr(self.t(f"{name}.phi")),
                              _ptr(self.t(f"{name}.{extra}")) if extra else None)
        w = self.t("weight")
        npu = self.t("npu")
        return DatasetS(self.n_events, F16 if self.content_dtype == "f16" else F32,
                        coll("jets", "btag" if self.t("jets.btag") is not None else None),
                        coll("muons", "iso"), coll("electrons", None),
                        _ptr(w) + 4 * self.e0 if w is not None else None,
                        _ptr(npu) + 4 * self.e0 if npu is not None else None)


def query_struct(q, keep: list) -> QueryS:
    """A datagen.Query as the C struct; host arrays it points to go into keep."""
    import numpy as np
    sc = np.ascontiguousarray(q.scales, np.float32)
    eds = [np.ascontiguousarray(e, np.float32) for e in q.edges()]
    keep += [sc] + eds
    qs = QueryS(q.mu_pt, q.mu_abseta, q.mu_iso, q.el_pt, q.el_abseta, q.jet_pt, q.jet_abseta,
                q.dr, q.btag, q.min_mu, q.min_jet, q.min_b, len(sc), sc.ctypes.data)
    for h in range(3):
        qs.edges[h] = eds[h].ctypes.data
        qs.nbins[h] = len(eds[h]) - 1

    def arr(a):
        a = np.ascontiguousarray(a, np.float32)
        keep.append(a)
        return a.ctypes.data
    if getattr(q, "pu", None) is not None:
        qs.pu_edges, qs.pu_contents, qs.pu_nbins = arr(q.pu[0]), arr(q.pu[1]), len(q.pu[0]) - 1
    if getattr(q, "sf", None) is not None:
        qs.sf_edges, qs.sf_contents, qs.sf_nbins = arr(q.sf[0]), arr(q.sf[1]), len(q.sf[0]) - 1
    if getattr(q, "jes", None) is not None:
        ee, pe, d = q.jes
        qs.jes_mode = 1
        qs.jes_eta_edges, qs.jes_pt_edges, qs.jes_delta = arr(ee), arr(pe), arr(d)
        qs.jes_n_eta, qs.jes_n_pt = len(ee) - 1, len(pe) - 1
    return qs


class Plan:
    """hepk_plan over device datasets and datagen.Query objects.

    shared_hist: all datasets accumulate into one set of histograms.
    reserve_bins: every query slot can later take (set_query) any query with
    at most that many bins per histogram.
    """

    def __init__(self, datasets: List[DeviceDataset], queries, tune: Optional[dict] = None,
                 shared_hist: bool = False, reserve_bins: int = 0, sumw2: bool = False, hist_arena_slots: int = 0):
        keep = []
        dsa = (DatasetS * len(datasets))(*[d.struct() for d in datasets])
        qa = (QueryS * len(queries))(*[query_struct(q, keep) for q in queries])
        opts = PlanOpts(Tune.of(tune) if tune is not None else Tune(0, 0, 0, 0),
                        1 if shared_hist else 0, reserve_bins, 1 if sumw2 else 0, hist_arena_slots)
        h = C.c_void_p()
        _call("hepk_plan_create_ex", dsa, len(datasets), qa, len(queries), C.byref(opts), C.byref(h))
        self.handle = h
        self.datasets = datasets
        self.queries = list(queries)
        self.shared = shared_hist
        n = C.c_int64()
        _call("hepk_plan_hist_slots", h, C.byref(n))
        self.n_slots = n.value
        t = Tune()
        _call("hepk_plan_get_tune", h, C.byref(t))
        self.tune = t.as_dict()

    def set_query(self, slot: int, q, stream=None, at: Optional[int] = None):
        """Install query q (None: idle) in a slot, ordered on the stream; with
        `at`, its histograms are placed from that slot of the buffers."""
        keep = []
        qs = C.byref(query_struct(q, keep)) if q is not None else None
        if at is None:
            _call("hepk_plan_set_query", self.handle, slot, qs, _stream(stream))
        else:
            _call("hepk_plan_set_query_at", self.handle, slot, qs, at, _stream(stream))
        self.queries[slot] = q

    def hist_offset(self, d: int, q: int, v: int, h: int):
        off, nb = C.c_int64(), C.c_int32()
        _call("hepk_plan_hist_offset", self.handle, d, q, v, h, C.byref(off), C.byref(nb))
        return off.value, nb.value

    def new_hists(self):
        import torch
        return (torch.zeros(self.n_slots, dtype=torch.float64, device="cuda"),
                torch.zeros(self.n_slots, dtype=torch.int64, device="cuda"))

    def run(self, sumw, counts, stream=None):
        _call("hepk_pipeline", self.handle, _ptr(sumw), _ptr(counts), _stream(stream))

    def run_w2(self, sumw, sumw2, counts, stream=None):
        """hepk_pipeline_w2: the pass that also sums squared weights."""
        _call("hepk_pipeline_w2", self.handle, _ptr(sumw), _ptr(sumw2), _ptr(counts), _stream(stream))

    def run_range(self, d0: int, nd: int, sumw, counts, stream=None):
        _call("hepk_pipeline_range", self.handle, d0, nd, _ptr(sumw), _ptr(counts), _stream(stream))

    def run_debug(self, sumw, counts, stream=None):
        """hepk_pipeline_debug: the pass plus every event's record; returns
        rec[d][q][v] = numpy structured array (EVENT_RECORD) of the dataset's
        events (None for idle slots).  Records never written keep state -1."""
        import numpy as np
        import torch
        n = C.c_int64()
        _call("hepk_plan_debug_layout", self.handle, 0, 0, None, None, C.byref(n))
        raw = torch.full((max(1, n.value) * 8,), -1, dtype=torch.int32, device="cuda")
        _call("hepk_pipeline_debug", self.handle, _ptr(sumw), _ptr(counts), _ptr(raw), _stream(stream))
        host_rec = raw.cpu().numpy().view(np.dtype(EVENT_RECORD))
        out = []
        for d, ds in enumerate(self.datasets):
            per_d = []
            for qi, q in enumerate(self.queries):
                if q is None:
                    per_d.append(None)
                    continue
                base, stride = C.c_int64(), C.c_int64()
                _call("hepk_plan_debug_layout", self.handle, d, qi, C.byref(base), C.byref(stride), None)
                per_d.append([host_rec[base.value + v * stride.value:base.value + v * stride.value + ds.n_events]
                              for v in range(q.n_scale)])
            out.append(per_d)
        return out

    def run_graph(self, sumw, counts, stream=None):
        _call("hepk_pipeline_graph", self.handle, _ptr(sumw), _ptr(counts), _stream(stream))

    def split(self, sumw, counts):
        """Host copies as hists[d][q][v][h] = (sumw, counts) numpy arrays."""
        s = sumw.cpu().numpy()
        c = counts.cpu().numpy().view("uint64")
        out = []
        for d in range(1 if self.shared else len(self.datasets)):
            per_d = []
            for qi, q in enumerate(self.queries):
                if q is None:
                    per_d.append(None)
                    continue
                per_q = []
                for v in range(q.n_scale):
                    per_v = []
                    for h in range(3):
                        off, nb = self.hist_offset(d, qi, v, h)
                        per_v.append((s[off:off + nb + 2].copy(), c[off:off + nb + 2].copy()))
                    per_q.append(per_v)
                per_d.append(per_q)
            out.append(per_d)
        return out

    def close(self):
        if self.handle:
            _call("hepk_plan_destroy", self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pipeline_noalloc(datasets: List[DeviceDataset], queries, sumw, counts, tune: Optional[dict] = None,
                     stream=None):
    """hepk_pipeline_noalloc: the fused pass without a plan (no device
    allocation); histograms laid out as a Plan over the same datasets and
    queries lays them out."""
    keep = []
    dsa = (DatasetS * len(datasets))(*[d.struct() for d in datasets])
    qa = (QueryS * len(queries))(*[query_struct(q, keep) for q in queries])
    t = C.byref(Tune.of(tune)) if tune is not None else None
    _call("hepk_pipeline_noalloc", dsa, len(datasets), qa, len(queries), t, _ptr(sumw), _ptr(counts),
          _stream(stream))


def host_dataset_struct(ds, keep: list) -> DatasetS:
    """A datagen.Dataset (host numpy arrays, or any objects with the same
    fields) as the C struct with HOST pointers; the arrays go into keep."""
    import numpy as np

    def p(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a)
        if a.size == 0:
            a = np.zeros(1, a.dtype)
        keep.append(a)
        return a.ctypes.data

    def coll(c, extra):
        if c is None:
            return Collection(None, None, None, None, None)
        return Collection(p(c.offsets), p(c.cols["pt"]), p(c.cols["eta"]), p(c.cols["phi"]),
                          p(c.cols[extra]) if extra and extra in c.cols else None)
    return DatasetS(ds.n_events, F16 if ds.content_dtype == "f16" else F32, coll(ds.jets, "btag"),
                    coll(ds.muons, "iso"), coll(ds.electrons, None), p(ds.weight),
                    p(getattr(ds, "npu", None)))


class Streamer:
    """hepk_streamer over a host dataset (datagen.Dataset: numpy arrays,
    possibly memory-mapped) for a list of datagen.Query; histograms laid out
    as a Plan over one dataset with the same queries."""

    def __init__(self, ds, queries, batch_events: int = 0, n_buffers: int = 0, host_threads: int = 0,
                 tune: Optional[dict] = None):
        self.keep = []
        self.ds = ds
        self.queries = list(queries)
        dss = host_dataset_struct(ds, self.keep)
        qa = (QueryS * len(queries))(*[query_struct(q, self.keep) for q in queries])
        self.keep += [dss, qa]
        opts = StreamOpts(batch_events, n_buffers, host_threads,
                          Tune.of(tune) if tune is not None else Tune(0, 0, 0, 0))
        h = C.c_void_p()
        _call("hepk_streamer_create", C.byref(dss), qa, len(queries), C.byref(opts), C.byref(h))
        self.handle = h
        n = C.c_int64()
        _call("hepk_streamer_hist_slots", h, C.byref(n))
        self.n_slots = n.value

    def new_hists(self):
        import torch
        return (torch.zeros(self.n_slots, dtype=torch.float64, device="cuda"),
                torch.zeros(self.n_slots, dtype=torch.int64, device="cuda"))

    def run(self, sumw, counts, stream=None):
        _call("hepk_stream_pass", self.handle, _ptr(sumw), _ptr(counts), _stream(stream))

    def close(self):
        if self.handle:
            _call("hepk_streamer_destroy", self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_cache_path() -> str:
    """Where launch-configuration search results are kept (HEPK_AUTOTUNE_CACHE,
    else ~/.cache/hepk/autotune.json)."""
    return os.environ.get("HEPK_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "hepk", "autotune.json"))


def workload_key(datasets, queries, device: Optional[str] = None) -> str:
    """Cache key of a launch-configuration search: the device (name,
    architecture, compute units) and the workload (events per dataset, content
    dtype, collections present, and per query its scales, binnings and
    lookups)."""
    import hashlib
    import json
    if device is None:
        import torch
        p = torch.cuda.get_device_properties(torch.cuda.current_device())
        device = f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"
    sig = {"events": [int(d.n_events) for d in datasets],
           "dtype": [d.content_dtype for d in datasets],
           "collections": [sorted(k for k in d.tensors if k.endswith(".offsets") or k.endswith(".btag"))
                           for d in datasets],
           "queries": [[int(q.n_scale), [len(e) - 1 for e in q.edges()], q.pu is not None, q.sf is not None,
                        q.jes is not None] for q in queries]}
    return device + "|" + hashlib.sha256(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:24]


def autotune(datasets: List[DeviceDataset], queries, reps: int = 5, stream=None, cache=None,
             device: Optional[str] = None):
    """Fastest launch configuration for these datasets and queries
    (hepk_autotune), and its median time in ms.  cache: a JSON file path (None:
    autotune_cache_path(); False: no cache) holding earlier results keyed by
    workload_key; a hit returns the stored result without searching."""
    import json
    import torch
    path = autotune_cache_path() if cache is None else cache
    key = workload_key(datasets, queries, device) if path else None
    table = {}
    if path and os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
        if key in table:
            hit = table[key]
            return dict(hit["tune"]), float(hit["ms"])
    keep = []
    dsa = (DatasetS * len(datasets))(*[d.struct() for d in datasets])
    qa = (QueryS * len(queries))(*[query_struct(q, keep) for q in queries])
    probe = Plan(datasets, queries)
    s = torch.zeros(probe.n_slots, dtype=torch.float64, device="cuda")
    c = torch.zeros(probe.n_slots, dtype=torch.int64, device="cuda")
    probe.close()
    best = Tune()
    ms = C.c_float()
    _call("hepk_autotune", dsa, len(datasets), qa, len(queries), _ptr(s), _ptr(c), reps,
          C.byref(best), C.byref(ms), _stream(stream))
    res = best.as_dict(), ms.value
    if path:
        table[key] = {"tune": res[0], "ms": res[1]}
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return res