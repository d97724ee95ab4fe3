#!/usr/bin/env python3
"""Throughput of the jagged-array analysis pass on one MI355X.

Workload (default): 1e7 synthetic events of the base schema (jets ~Poisson(5)
capped at 20, muons ~Poisson(1.5) capped at 8, float32 content, int64
offsets, seed 0), all columns resident in HBM.  One step = one full analysis
pass (muon and jet selection, jet-muon Delta-R cleaning, per-event counts,
H_T and leading pt, event selection, three weighted histograms) by the fused
persistent kernel (hepk_pipeline).  The same pass as a chain of ~11
single-purpose kernel calls (the per-kernel pipeline) is timed beside it.

Prints ONE JSON line.  `value` is fused events/s; `roofline` is the fused
kernel's achieved HBM bandwidth from its algorithmic bytes (the input columns
the pass must read, mass columns excluded) over its average launch time,
measured with HIP events on the launch stream; `cpu_baseline` is the CPU
oracle on one host core over a bounded sample of the same workload.

Further sections on the same line (each skippable):
  primitives  each single-purpose entry point of the per-kernel chain timed
            alone on the same 1e7 events: algorithmic bytes / HIP-event time
            against the HBM peak;
  extended  5e7 events, float16 content widened in registers, electrons,
            jet b-tag, 20 jet-energy-scale variations -> 60 histograms/pass;
  batch     64 datasets of log-uniform sizes in [1e4, 5e6] in one persistent
            launch replayed from a HIP graph, with the launch-configuration
            sweep (block, events per thread, LDS vs global histograms);
  serving   2e8 events resident, Poisson stream of queries at 50/s with
            random cuts and binnings, continuous batching over a circular
            chunk scan: p50/p99 latency and query-events/s, plus closed-loop
            throughput of the fused server vs the per-kernel pipeline;
  positional  get_in_offsets, opposite-sign pairs, compaction, four-momenta
            and the top-quark triplet search on the 1e7 events;
  lookups   the lookup primitives and the fused pass with lookup event
            weights, 20 interpolated jet-energy shifts and squared weights
            over 5e7 float16 events;
  streaming 5e7 events held in host memory, streamed in batches with copies
            overlapping the passes, against a plain host-to-device copy.
The extended, lookup, batch and serving inputs are drawn on the GPU
(datagen.make_dataset_device); the streaming input on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pipeline_fused_1e7_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_1906_06242_amd/csrc/common.hpp", "paper_1906_06242_amd/csrc/lookup.hpp",
              "paper_1906_06242_amd/csrc/pipeline_kernel.hpp", "paper_1906_06242_amd/csrc/plan.hpp",
              "paper_1906_06242_amd/csrc/pipeline.hip", "paper_1906_06242_amd/csrc/pipeline_ms.hip"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_traffic(events: int):
    """HBM bytes per fused launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    passes (scaled by a plain copy of known size), or None when they were taken
    for another workload or an older version of the kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        tr = json.load(f)
    if tr.get("events") != events or tr.get("source_sha256") != kernel_sources_sha256():
        return None
    return tr.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ds, q, reps: int):
    """The oracle (one thread, as it stands) on the same events, pinned to one
    host core; median pass time."""
    from oracle import ref
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            ref.pipeline(ds, [q])
            times.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, old)
    med = statistics.median(times)
    return {"value": ds.n_events / med, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} passes over the full {ds.n_events:.0e}-event workload, median "
                      f"{med:.2f} s/pass (single-threaded C pinned to host core {core} of the GPU box)",
            "cpu_model": cpu_model()}


def time_flushed(fn, reps: int, stream, flush):
    """Median HIP-event duration (ms) of fn, the last-level cache refilled by a
    read of `flush` (>= 512 MB, clean lines: nothing to write back during the
    timed launch) before each repetition."""
    import torch
    fn()
    ms = []
    sink = torch.empty((), dtype=flush.dtype, device=flush.device)
    for _ in range(reps):
        torch.sum(flush, dim=0, out=sink)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    return statistics.median(ms)


def streaming_ceiling(stream, flush) -> dict:
    """What plain streaming reaches on this GPU: hepk_stream_read (16-byte
    loads, nothing else) and torch's sum over 1 GiB (read only), and a 1 GiB
    device copy (read + write)."""
    import torch
    from paper_1906_06242_amd import hepk as H
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    nb = x.numel() * 4
    h_ms = time_flushed(lambda: H.stream_read(x, sink), 10, stream, flush)
    r_ms = time_flushed(lambda: x.sum(), 10, stream, flush)
    c_ms = time_flushed(lambda: y.copy_(x), 10, stream, flush)
    del x, y
    return {"read_GBps": nb / (h_ms * 1e-3) / 1e9, "torch_sum_GBps": nb / (r_ms * 1e-3) / 1e9,
            "copy_GBps": 2 * nb / (c_ms * 1e-3) / 1e9,
            "what": "hepk_stream_read and torch sum over 1 GiB float32 (read), 1 GiB device copy (read + write), "
                    "median of 10, last-level cache refilled by a 512 MB read before each"}


def time_steps(fn, steps: int, warmup: int, stream):
    """Run warmup + timed steps; per-step HIP-event durations (ms) and wall ms."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return [a.elapsed_time(b) for a, b in ev], wall


def warm_up(fn, warmup: int, min_ms: float = 0.0) -> int:
    """warmup untimed steps, continued until min_ms of them have run; returns
    how many ran."""
    import torch
    done = 0
    t0 = time.perf_counter()
    while done < warmup or (time.perf_counter() - t0) * 1e3 < min_ms:
        fn()
        done += 1
        if done % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return done


def time_back_to_back(fn, steps: int, warmup: int, stream, min_warm_ms: float = 0.0):
    """warmup untimed steps (at least min_warm_ms of them), then `steps`
    launches back to back between one pair of HIP events on the launch stream
    (no event between launches), the whole bracketed by synchronisation.
    Returns (event ms per launch, wall ms per step)."""
    import torch
    warm_up(fn, warmup, min_warm_ms)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return a.elapsed_time(b) / steps, wall / steps


def dev_bytes_read(t: dict) -> int:
    """Algorithmic bytes of one pass over an on-device dataset (mass columns excluded)."""
    b = 0
    for k, v in t.items():
        if hasattr(v, "element_size") and not k.endswith(".mass"):
            b += v.numel() * v.element_size()
    return b


def time_plan(run, steps: int, warmup: int = 2, min_warm_ms: float = 0.0):
    """(event ms per launch, wall ms per step) of `steps` back-to-back runs
    after `warmup` runs (continued for at least min_warm_ms)."""
    import torch
    return time_back_to_back(run, steps, warmup, torch.cuda.current_stream(), min_warm_ms)


def spot_check(dd_all: dict, e0: int, e1: int, queries, tune=None) -> bool:
    """Fused pass over events [e0, e1) of a device dataset vs the oracle on a host copy."""
    import numpy as np
    from oracle import ref
    from paper_1906_06242_amd import datagen
    from paper_1906_06242_amd import hepk as H
    view = H.DeviceDataset.from_tensors(dd_all).view(e0, e1)
    plan = H.Plan([view], queries, tune)
    s, c = plan.new_hists()
    plan.run(s, c)
    got = plan.split(s, c)[0]
    plan.close()
    want = ref.pipeline(datagen.host_slice(dd_all, e0, e1), queries)
    ok = True
    for qi, qq in enumerate(queries):
        for v in range(qq.n_scale):
            for h in range(3):
                gs, gc = got[qi][v][h]
                ws, wc = want[qi][v][h]
                ok &= bool(np.array_equal(gc, wc) and np.all(np.abs(gs - ws) <= 1e-5 * np.abs(ws)))
    return ok


def section_primitives(dd, q, stream, reps: int = 10) -> dict:
    """Each entry point of the per-kernel chain alone: median HIP-event time,
    algorithmic bytes (inputs read + outputs written), fraction of HBM peak."""
    import torch
    from paper_1906_06242_amd import hepk as H
    t = dd.t
    n, mm, mj = dd.n_events, t("muons.pt").numel(), t("jets.pt").numel()
    ob = 8 * (n + 1)  # one offsets array
    msel = H.select([(t("muons.pt"), H.GT, q.mu_pt), (t("muons.eta"), H.ABS_LT, q.mu_abseta),
                     (t("muons.iso"), H.LT, q.mu_iso)], mm)
    _, _, clean = H.match_dr(t("jets.offsets"), t("jets.eta"), t("jets.phi"), t("muons.offsets"),
                             t("muons.eta"), t("muons.phi"), q.dr, mask_b=msel, want=("clean",))
    jsel = H.select([(t("jets.pt"), H.GT, q.jet_pt), (t("jets.eta"), H.ABS_LT, q.jet_abseta)], mj,
                    mask_in=clean)
    nmu = H.reduce(H.COUNT, t("muons.offsets"), obj_mask=msel)
    njet = H.reduce(H.COUNT, t("jets.offsets"), obj_mask=jsel)
    ht = H.reduce(H.SUM, t("jets.offsets"), t("jets.pt"), obj_mask=jsel)
    passed = H.select([(nmu, H.GE, q.min_mu), (njet, H.GE, q.min_jet)], n)
    e = torch.from_numpy(q.edges_ht.astype("float32")).to("cuda")
    hs = torch.zeros(len(e) + 1, dtype=torch.float64, device="cuda")
    hc = torch.zeros(len(e) + 1, dtype=torch.int64, device="cuda")
    o_mask, o_i32 = torch.empty(mj, dtype=torch.uint8, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda")
    o_f32 = torch.empty(n, dtype=torch.float32, device="cuda")
    cases = {
        "select (muons, 3 cuts)": (lambda: H.select([(t("muons.pt"), H.GT, q.mu_pt),
                                                     (t("muons.eta"), H.ABS_LT, q.mu_abseta),
                                                     (t("muons.iso"), H.LT, q.mu_iso)], mm, out=o_mask[:mm]),
                                   13 * mm),
        "select (jets, 2 cuts + mask)": (lambda: H.select([(t("jets.pt"), H.GT, q.jet_pt),
                                                           (t("jets.eta"), H.ABS_LT, q.jet_abseta)], mj,
                                                          mask_in=clean, out=o_mask), 10 * mj),
        "select (events, 2 int32 cuts)": (lambda: H.select([(nmu, H.GE, q.min_mu), (njet, H.GE, q.min_jet)], n,
                                                           out=o_mask[:n]), 9 * n),
        "match_dr (jets vs selected muons, clean mask)": (
            lambda: H.match_dr(t("jets.offsets"), t("jets.eta"), t("jets.phi"), t("muons.offsets"),
                               t("muons.eta"), t("muons.phi"), q.dr, mask_b=msel, want=("clean",)),
            2 * ob + 8 * mj + 9 * mm + mj),
        "reduce COUNT (jets, mask)": (lambda: H.reduce(H.COUNT, t("jets.offsets"), obj_mask=jsel, out=o_i32),
                                      ob + mj + 4 * n),
        "reduce SUM (jet pt, mask)": (lambda: H.reduce(H.SUM, t("jets.offsets"), t("jets.pt"), obj_mask=jsel,
                                                       out=o_f32), ob + 5 * mj + 4 * n),
        "reduce MAX (jet pt, mask)": (lambda: H.reduce(H.MAX, t("jets.offsets"), t("jets.pt"), obj_mask=jsel,
                                                       out=o_f32), ob + 5 * mj + 4 * n),
        "hist_fill (H_T, weights, event mask)": (lambda: H.hist_fill(ht, e, hs, hc, w=t("weight"),
                                                                      evt_mask=passed), 9 * n),
    }
    res = {}
    for name, (fn, nbytes) in cases.items():
        ms = time_back_to_back(fn, reps, 2, stream)[0]
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms": ms, "bytes": int(nbytes), "GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
        log(f"primitive {name}: {ms * 1e3:.1f} us, {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.0f}% of HBM peak)")
    return res


def section_lookups(args) -> dict:
    """Lookup corrections: the per-element lookup primitives, and the fused pass
    with lookup event weights and 20 interpolated jet-energy shifts (and the
    squared weights) over the extended schema."""
    import torch
    from paper_1906_06242_amd import datagen
    from paper_1906_06242_amd import hepk as H
    n = 50_000_000
    t = datagen.with_pileup_device(datagen.make_dataset_device(0, n, extended=True, content_dtype="f16"), 0)
    torch.cuda.synchronize()
    q = datagen.lookup_query()
    stream = torch.cuda.current_stream()
    res = {"workload": "5e7 events, f16 content, pileup column, pileup and muon scale-factor weights, "
                       "20 interpolated jet-energy shifts, 60 histograms with squared weights"}
    # primitives on the same columns
    pe, pc = (torch.from_numpy(a).cuda() for a in q.pu)
    se, sc = (torch.from_numpy(a).cuda() for a in q.sf)
    ee, pte, dl = (torch.from_numpy(a).cuda() for a in q.jes)
    mpt, jpt, jeta = t["muons.pt"], t["jets.pt"], t["jets.eta"]
    o_m = torch.empty(mpt.numel(), dtype=torch.float32, device="cuda")
    o_j = torch.empty(jpt.numel(), dtype=torch.float32, device="cuda")
    o_e = torch.empty(n, dtype=torch.float32, device="cuda")
    prim = {
        "get_bin_contents (pileup, per event)": (lambda: H.get_bin_contents(t["npu"], pe, pc, out=o_e), 8 * n),
        "get_bin_contents (muon scale factors)": (lambda: H.get_bin_contents(mpt, se, sc, out=o_m),
                                                  6 * mpt.numel()),
        "interp (muon scale factors)": (lambda: H.interp(mpt, se, sc, out=o_m), 6 * mpt.numel()),
        "jes_delta (jets, |eta| x pt table)": (lambda: H.jes_delta(jpt, jeta, ee, pte, dl, out=o_j),
                                               8 * jpt.numel()),
    }
    res["primitives"] = {}
    for name, (fn, nbytes) in prim.items():
        ms = time_back_to_back(fn, 20, 3, stream)[0]
        res["primitives"][name] = {"ms": ms, "bytes": nbytes, "GBps": nbytes / (ms * 1e-3) / 1e9,
                                   "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"lookups: {name}: {ms * 1e3:.1f} us, {nbytes / (ms * 1e-3) / 1e9:.0f} GB/s")
    del o_m, o_j, o_e
    dd = H.DeviceDataset.from_tensors(t)
    plan = H.Plan([dd], [q])
    s, c = plan.new_hists()
    w2 = torch.zeros_like(s)
    kern_ms, step_ms = time_plan(lambda: plan.run_w2(s, w2, c), 10, 3, args.warm_ms)
    alg = dev_bytes_read(t)
    res.update({"events_per_s": n / (step_ms * 1e-3), "ms_per_step": step_ms, "kernel_ms": kern_ms,
                "bytes_read_per_pass": alg, "achieved_GBps": alg / (kern_ms * 1e-3) / 1e9,
                "hbm_frac": alg / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "tune": plan.tune})
    plan.close()
    res["parity_spot_check"] = spot_check(t, 2_345_678, 2_365_678, [q])
    log(f"lookups: fused {step_ms:.3f} ms/step, {res['achieved_GBps']:.0f} GB/s, parity {res['parity_spot_check']}")
    del t, dd
    torch.cuda.empty_cache()
    return res


def section_positional(dd, ds, q, stream) -> dict:
    """Positional kernels, compaction and the top-quark triplet search on the
    1e7-event workload: HIP-event time per call and algorithmic bytes (inputs
    read + outputs written); the triplet search also in float32 operations."""
    import torch
    from paper_1906_06242_amd import hepk as H
    t = dd.t
    n, mj, mm = dd.n_events, t("jets.pt").numel(), t("muons.pt").numel()
    jsel = H.select([(t("jets.pt"), H.GT, q.jet_pt), (t("jets.eta"), H.ABS_LT, q.jet_abseta)], mj)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    charge = (torch.randint(0, 2, (mm,), generator=g, device="cuda", dtype=torch.int32) * 2 - 1).contiguous()
    cnt, offo = H.reduce(H.COUNT, t("jets.offsets"), obj_mask=jsel, want_offsets=True)
    n_sel = int(offo[-1].item())
    out_c = torch.empty(max(1, n_sel), dtype=torch.float32, device="cuda")
    jmass = torch.from_numpy(ds.jets.cols["mass"]).cuda()  # the resident dataset skips the unread masses
    p4 = H.p4(t("jets.pt"), t("jets.eta"), t("jets.phi"), jmass)
    ob = 8 * (n + 1)
    cases = {
        "get_in_offsets (leading selected jet pt)": (
            lambda: H.get_in_offsets(t("jets.offsets"), t("jets.pt"), n=0, obj_mask=jsel), ob + mj + 4 * n + 8 * n),
        "select_opposite_sign (muons)": (
            lambda: H.select_opposite_sign(t("muons.offsets"), t("muons.pt"), charge), ob + 9 * mm),
        "compact (selected jet pt)": (
            lambda: H.compact(t("jets.offsets"), t("jets.pt"), offo, n_sel, obj_mask=jsel, out=out_c),
            2 * ob + mj + 4 * mj + 4 * n_sel),
        "p4 (jets)": (lambda: H.p4(t("jets.pt"), t("jets.eta"), t("jets.phi"), jmass), 32 * mj),
        "best_triplet (selected jets, 172 GeV)": (
            lambda: H.best_triplet(t("jets.offsets"), *p4, obj_mask=jsel), ob + 17 * mj + 16 * n),
    }
    res = {}
    for name, (fn, nbytes) in cases.items():
        ms = time_back_to_back(fn, 20, 3, stream)[0]
        res[name] = {"ms": ms, "bytes": int(nbytes), "GBps": nbytes / (ms * 1e-3) / 1e9,
                     "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"positional: {name}: {ms * 1e3:.1f} us, {nbytes / (ms * 1e-3) / 1e9:.0f} GB/s")
    # the triplet search's float32 work: triplets per event from the selected-jet counts
    k = cnt.to(torch.float64)
    triplets = float((k * (k - 1) * (k - 2) / 6).sum().item())
    flops = 24.0 * triplets  # 12 adds, 4 multiplies, 3 subtractions, sqrt, |.|, compare per triplet
    ms = res["best_triplet (selected jets, 172 GeV)"]["ms"]
    res["best_triplet (selected jets, 172 GeV)"].update(
        {"triplets": triplets, "flops_per_call": flops, "TFLOPs": flops / (ms * 1e-3) / 1e12,
         "valu_frac": flops / (ms * 1e-3) / 1e12 / 157.3})
    return res


def section_streaming(args) -> dict:
    """Out-of-core passes: 5e7 base-schema events in host memory streamed to
    the device in batches of 2^22 events (copies overlapping the passes), from
    pageable and from pinned host memory, against a plain pinned host-to-device
    copy of the same bytes."""
    import torch
    from paper_1906_06242_amd import datagen
    from paper_1906_06242_amd import hepk as H
    n = args.stream_events
    t0 = time.time()
    ds = datagen.make_dataset(7, n)
    log(f"streaming: generated {n} host events in {time.time() - t0:.1f} s")
    q = datagen.Query()
    nbytes = ds.nbytes_read()
    res = {"workload": f"{n:.0e} base-schema events in host memory, batches of 2^22 events, 2 device slots",
           "bytes_per_pass": nbytes}
    # the link: one pinned host-to-device copy of 1 GiB
    hsrc = torch.empty(1 << 28, dtype=torch.float32).pin_memory()
    ddst = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    ddst.copy_(hsrc, non_blocking=True)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(3):
        ddst.copy_(hsrc, non_blocking=True)
    b.record()
    torch.cuda.synchronize()
    res["h2d_copy_GBps"] = 3 * (1 << 30) / (a.elapsed_time(b) * 1e-3) / 1e9
    del hsrc, ddst
    for kind in ("pageable", "pinned"):
        src = ds
        keep = []
        if kind == "pinned":
            def pin(name, arr):
                tt = torch.from_numpy(np.ascontiguousarray(arr)).pin_memory()
                keep.append(tt)
                return tt.numpy()

            def coll(name, c):
                return datagen.Collection(pin("", c.offsets), {k: pin("", v) for k, v in c.cols.items()})
            src = datagen.Dataset(ds.n_events, coll("jets", ds.jets), coll("muons", ds.muons), pin("", ds.weight))
        st = H.Streamer(src, [q], batch_events=1 << 22, n_buffers=2)
        s, c = st.new_hists()
        st.run(s, c)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(2):
            st.run(s, c)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - w0) / 2
        st.close()
        res[kind] = {"s_per_pass": sec, "events_per_s": n / sec, "GBps": nbytes / sec / 1e9,
                     "of_h2d_copy": nbytes / sec / 1e9 / res["h2d_copy_GBps"]}
        log(f"streaming ({kind}): {sec * 1e3:.1f} ms/pass, {n / sec:.3e} events/s, {nbytes / sec / 1e9:.1f} GB/s")
        del keep
    return res


def section_extended(args) -> dict:
    import torch
    from paper_1906_06242_amd import datagen
    from paper_1906_06242_amd import hepk as H
    n = 50_000_000
    t0 = time.time()
    t = datagen.make_dataset_device(0, n, extended=True, content_dtype="f16")
    torch.cuda.synchronize()
    log(f"extended: generated {n} events on device in {time.time() - t0:.1f} s")
    q = datagen.extended_query()
    dd = H.DeviceDataset.from_tensors(t)
    plan = H.Plan([dd], [q])
    s, c = plan.new_hists()
    kern_ms, step_ms = time_plan(lambda: plan.run(s, c), 10, 2, args.warm_ms)
    alg = dev_bytes_read(t)
    res = {"workload": "5e7 events, f16 content, jets+muons+electrons, b-tag, 20 JES scales, 60 histograms",
           "events_per_s": n / (step_ms * 1e-3), "ms_per_step": step_ms, "kernel_ms": kern_ms,
           "bytes_read_per_pass": alg, "bytes_per_event": alg / n,
           "achieved_GBps": alg / (kern_ms * 1e-3) / 1e9, "hbm_frac": alg / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "tune": plan.tune, "histograms": 60}
    plan.close()
    res["parity_spot_check"] = spot_check(t, 1_234_567, 1_264_567, [q])
    log(f"extended: {step_ms:.3f} ms/step, {res['achieved_GBps']:.0f} GB/s, parity {res['parity_spot_check']}")
    del t, dd
    torch.cuda.empty_cache()
    return res


def section_batch(args) -> dict:
    import torch
    from paper_1906_06242_amd import datagen
    from paper_1906_06242_amd import hepk as H
    sizes = datagen.batch_sizes(0)
    t0 = time.time()
    ts = [datagen.make_dataset_device(1000 + d, int(n)) for d, n in enumerate(sizes)]
    torch.cuda.synchronize()
    n_all = int(sizes.sum())
    log(f"batch: generated {len(sizes)} datasets, {n_all} events, in {time.time() - t0:.1f} s")
    dds = [H.DeviceDataset.from_tensors(t) for t in ts]
    q = datagen.Query()
    alg = sum(dev_bytes_read(t) for t in ts)
    sweep = []
    # the sweep starts from the clocks of a GPU that has been busy (a pass run
    # for args.warm_ms first), like every later timing here
    plan = H.Plan(dds, [q])
    s, c = plan.new_hists()
    warm_up(lambda: plan.run(s, c), 2, args.warm_ms)
    plan.close()
    for blk in (256, 512):
        for evpt in (1, 2):
            for hm in (0, 1):
                tn = {"block": blk, "ev_per_thread": evpt, "hist_mode": hm}
                plan = H.Plan(dds, [q], tn)
                s, c = plan.new_hists()
                kern_ms, _ = time_plan(lambda: plan.run(s, c), 5, 1)
                sweep.append({"tune": tn, "kernel_ms": kern_ms})
                plan.close()
    best, best_ms = H.autotune(dds, [q], reps=5, cache=False)  # always search here (its time is reported)
    plan = H.Plan(dds, [q], best)
    s, c = plan.new_hists()
    strict_ms, _ = time_plan(lambda: plan.run_graph(s, c), 10)
    kern_ms, step_ms = time_plan(lambda: plan.run_graph(s, c), 20, 2, args.warm_ms)
    res = {"workload": f"{len(sizes)} datasets, log-uniform sizes in [1e4, 5e6], {n_all} events, one graph launch",
           "events": n_all, "events_per_s": n_all / (step_ms * 1e-3), "ms_per_step": step_ms,
           "kernel_ms": kern_ms, "bytes_read_per_pass": alg,
           "achieved_GBps": alg / (kern_ms * 1e-3) / 1e9, "hbm_frac": alg / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "autotuned": best, "autotune_ms": best_ms, "sweep": sweep,
           "after_exact_warmup": {"kernel_ms": strict_ms,
                                  "hbm_frac": alg / (strict_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "what": "10 graph launches right after 2 warm-up launches"},
           "timing": f"20 graph launches back to back after at least {args.warm_ms:.0f} ms of warm-up launches"}
    plan.close()
    res["parity_spot_check"] = spot_check(ts[5], 0, min(40000, int(sizes[5])), [q])
    log(f"batch: {step_ms:.3f} ms/step, {res['achieved_GBps']:.0f} GB/s, best {best}")
    del ts, dds
    torch.cuda.empty_cache()
    return res


def section_serving(args) -> dict:
    import torch
    from paper_1906_06242_amd import datagen
    from paper_1906_06242_amd import hepk as H
    from paper_1906_06242_amd import plain
    from paper_1906_06242_amd.serve import GpuBackend, Server, percentile
    n = 200_000_000
    t0 = time.time()
    t = datagen.make_dataset_device(0, n)
    torch.cuda.synchronize()
    log(f"serving: generated {n} events on device in {time.time() - t0:.1f} s")
    dd = H.DeviceDataset.from_tensors(t)
    stored = sum(v.numel() * v.element_size() for v in t.values() if hasattr(v, "numel"))
    qs = datagen.draw_queries(1, args.serve_queries, qps=50.0)
    be = GpuBackend(dd, n_chunks=16, n_slots=8)
    # warm-up: a few queries closed loop
    Server(be).run_closed(datagen.draw_queries(2, 4))
    srv = Server(be)
    w0 = time.perf_counter()
    done = srv.run_stream(qs)
    wall = time.perf_counter() - w0
    lat = [x.latency * 1e3 for x in done]
    parts = {k: [getattr(x, k) * 1e3 for x in done] for k in ("queue_wait", "scan", "copy_out")}
    res = {"workload": f"{n:.0e} events resident ({stored / 1e9:.1f} GB), {len(qs)} queries, Poisson 50/s, "
                       "16 chunks, 8 query slots, 64 MB histogram arena",
           "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99), "max_ms": max(lat),
           "breakdown_ms": {k: {"p50": percentile(v, 50), "p99": percentile(v, 99)} for k, v in parts.items()},
           "queries": len(done), "wall_s": wall, "query_events_per_s": len(done) * n / wall,
           "launches": srv.launches}
    # closed loop: all queries waiting, fused co-batched server vs per-kernel pipeline per query
    qc = datagen.draw_queries(3, 32)
    srv = Server(be)
    w0 = time.perf_counter()
    srv.run_closed(qc)
    torch.cuda.synchronize()
    res["saturated_query_events_per_s"] = len(qc) * n / (time.perf_counter() - w0)
    be.close()
    qp = qc[:3]
    plain.run(dd, qp[0])
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for x in qp:
        plain.run(dd, x)
    torch.cuda.synchronize()
    res["plain_query_events_per_s"] = len(qp) * n / (time.perf_counter() - w0)
    res["served_over_plain"] = res["saturated_query_events_per_s"] / res["plain_query_events_per_s"]
    log(f"serving: p50 {res['p50_ms']:.2f} ms, p99 {res['p99_ms']:.2f} ms, "
        f"saturated {res['saturated_query_events_per_s']:.3e} vs plain {res['plain_query_events_per_s']:.3e}")
    del t, dd
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--warm-ms", type=float, default=200.0,
                    help="warm-up passes continue until this many ms of them have run")
    ap.add_argument("--events", type=int, default=10_000_000)
    ap.add_argument("--no-plain", action="store_true", help="skip the per-kernel pipeline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-reps", type=int, default=7)
    ap.add_argument("--tune", type=str, default="", help="JSON launch configuration")
    ap.add_argument("--sections", type=str,
                    default="primitives,positional,extended,lookups,batch,serving,streaming",
                    help="comma list of extra sections to run (primitives, positional, extended, lookups, batch, "
                         "serving, streaming) or 'none'")
    ap.add_argument("--stream-events", type=int, default=50_000_000)
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (scale for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1906_06242_amd import datagen
    from paper_1906_06242_amd import hepk as H
    from paper_1906_06242_amd import plain

    assert torch.cuda.is_available(), "needs a HIP device"
    H.load()
    t0 = time.time()
    ds = datagen.make_dataset(0, args.events)
    log(f"generated {args.events} events in {time.time() - t0:.1f} s")
    q = datagen.Query()
    dd = H.DeviceDataset(ds)
    torch.cuda.synchronize()
    alg_bytes = ds.nbytes_read()
    tune = json.loads(args.tune) if args.tune else None
    plan = H.Plan([dd], [q], tune)
    sumw, counts = plan.new_hists()
    stream = torch.cuda.current_stream()

    sections = [x for x in args.sections.split(",") if x and x != "none"]
    early = {}
    # the per-kernel chain and the single-purpose kernels, on the same resident events
    if not args.no_plain:
        plain_ms, plain_wall = time_steps(lambda: plain.run(dd, q), max(5, args.steps // 5), 2, stream)
        early["plain_step"] = plain_wall / max(5, args.steps // 5)
        log(f"plain: {early['plain_step']:.3f} ms/step")
    if "primitives" in sections:
        early["primitives"] = section_primitives(dd, q, stream)
    if "positional" in sections:
        early["positional"] = section_positional(dd, ds, q, stream)

    # the strict reading first: W warm-up passes straight after other work,
    # then K timed -- on a GPU coming from idle or from lighter work this
    # catches its clocks still settling (per-pass time rises by up to 25% over
    # the first tens of ms of sustained passes, then falls below the first
    # passes' time)
    strict_ms, _ = time_back_to_back(lambda: plan.run(sumw, counts), args.steps, args.warmup, stream)
    # the timed region: W warm-up passes continued for at least 200 ms of
    # passes (the settled state a long job runs in), then K launches back to
    # back between one event pair
    n_warm = warm_up(lambda: plan.run(sumw, counts), args.warmup, args.warm_ms)
    kern_ms, ms_step = time_back_to_back(lambda: plan.run(sumw, counts), args.steps, 0, stream)
    value = args.events / (ms_step * 1e-3)
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    log(f"fused: {ms_step:.3f} ms/step wall, {kern_ms:.3f} ms/launch on the stream, {achieved:.0f} GB/s")
    # the same launches each bracketed by its own event pair: the difference is
    # the cost of the event records between launches
    each_ms, _ = time_steps(lambda: plan.run(sumw, counts), args.steps, 2, stream)
    each_ms = statistics.mean(each_ms)
    # a long run: 300 back-to-back passes, the last 100 timed
    for _ in range(200):
        plan.run(sumw, counts)
    steady_ms, _ = time_back_to_back(lambda: plan.run(sumw, counts), 100, 0, stream)
    log(f"fused, settled (passes 201-300 of a run): {steady_ms:.3f} ms/launch, "
        f"{alg_bytes / (steady_ms * 1e-3) / 1e9:.0f} GB/s")

    traffic = kernel_traffic(args.events)
    # the same launch with the 256 MB last-level cache refilled by other data
    # before each of 10 repetitions (median), and what plain streaming reaches
    flush = torch.ones(1 << 27, dtype=torch.float32, device="cuda")  # 512 MB
    flushed_ms = time_flushed(lambda: plan.run(sumw, counts), 10, stream, flush)
    ceiling = streaming_ceiling(stream, flush)
    del flush
    log(f"fused, cache flushed: {flushed_ms:.3f} ms/launch, {alg_bytes / (flushed_ms * 1e-3) / 1e9:.0f} GB/s; "
        f"streaming read {ceiling['read_GBps']:.0f} GB/s, copy {ceiling['copy_GBps']:.0f} GB/s")

    out = {
        "metric": "events/s and % HBM roofline, fused vs plain pipeline; query p50/p99 latency",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator; CMS Open Data not available)",
        "config": {"workload": f"base schema, {args.events:.0e} events resident in HBM, "
                               "one fused analysis pass per step",
                   "events": args.events, "seed": 0, "tune": plan.tune,
                   "bytes_read_per_pass": alg_bytes, "bytes_per_event": alg_bytes / args.events},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "warmup_passes_run": n_warm,
        "warmup_min_ms": args.warm_ms,
        "after_exact_warmup": {"ms_per_launch": strict_ms, "achieved": alg_bytes / (strict_ms * 1e-3) / 1e9,
                               "frac": alg_bytes / (strict_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "what": "K passes right after exactly W warm-up passes"},
        "launch_timing": {"back_to_back_ms_per_launch": kern_ms, "wall_ms_per_step": ms_step,
                          "host_gap_ms_per_step": ms_step - kern_ms,
                          "event_pair_per_launch_ms": each_ms,
                          "what": "back_to_back: K launches between one HIP event pair on the launch stream "
                                  "(roofline.achieved uses it); wall: host clock over the same K steps; "
                                  "event_pair: each launch between its own event pair (records in between)"},
        "settled": {"ms_per_launch": steady_ms, "achieved": alg_bytes / (steady_ms * 1e-3) / 1e9,
                    "unit": "GB/s", "frac": alg_bytes / (steady_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "what": "passes 201-300 of 300 back-to-back passes, one event pair around the last 100"},
        "roofline_cache_flushed": {"ms_per_launch": flushed_ms,
                                   "achieved": alg_bytes / (flushed_ms * 1e-3) / 1e9, "unit": "GB/s",
                                   "frac": alg_bytes / (flushed_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "streaming_ceiling": ceiling,
    }

    if not args.no_plain:
        p_step = early["plain_step"]
        out["plain"] = {"events_per_s": args.events / (p_step * 1e-3), "ms_per_step": p_step,
                        "hbm_frac_vs_algorithmic": alg_bytes / (p_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "launches_per_step": 11}
        out["fused_over_plain"] = p_step / ms_step
    for k in ("primitives", "positional"):
        if k in early:
            out[k] = early[k]
    plan.close()
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(ds, q, args.cpu_reps)
        out["cpu_baseline"]["host_nproc"] = os.cpu_count()
        out["cpu_baseline"]["gpu_over_one_core"] = value / out["cpu_baseline"]["value"]
        log(f"cpu oracle: {out['cpu_baseline']['value']:.3e} events/s")
    del dd, ds
    torch.cuda.empty_cache()
    if "extended" in sections:
        out["extended"] = section_extended(args)
    if "lookups" in sections:
        out["lookups"] = section_lookups(args)
    if "batch" in sections:
        out["batch"] = section_batch(args)
    if "serving" in sections:
        out["serving"] = section_serving(args)
    if "streaming" in sections:
        out["streaming"] = section_streaming(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
