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
    for f in ("paper_1906_06242_amd/csrc/pipeline.hip", "paper_1906_06242_amd/csrc/common.hpp"):
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


def cpu_baseline(ds, q, reps: int):
    """The oracle (one thread, as it stands) on the same events; median pass time."""
    from oracle import ref
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ref.pipeline(ds, [q])
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    return {"value": ds.n_events / med, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} passes over the full {ds.n_events:.0e}-event workload, median "
                      f"{med:.2f} s/pass (single-threaded C, host core of the GPU box)"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--events", type=int, default=10_000_000)
    ap.add_argument("--no-plain", action="store_true", help="skip the per-kernel pipeline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-reps", type=int, default=4)
    ap.add_argument("--tune", type=str, default="", help="JSON launch configuration")
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

    fused_ms, fused_wall = time_steps(lambda: plan.run(sumw, counts), args.steps, args.warmup, stream)
    ms_step = fused_wall / args.steps
    kern_ms = statistics.mean(fused_ms)
    value = args.events / (ms_step * 1e-3)
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    log(f"fused: {ms_step:.3f} ms/step wall, {kern_ms:.3f} ms/launch, {achieved:.0f} GB/s")

    traffic = kernel_traffic(args.events)

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
    }

    if not args.no_plain:
        plain_ms, plain_wall = time_steps(lambda: plain.run(dd, q), max(5, args.steps // 5), 2, stream)
        p_step = plain_wall / max(5, args.steps // 5)
        out["plain"] = {"events_per_s": args.events / (p_step * 1e-3), "ms_per_step": p_step,
                        "hbm_frac_vs_algorithmic": alg_bytes / (p_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "launches_per_step": 11}
        out["fused_over_plain"] = p_step / ms_step
        log(f"plain: {p_step:.3f} ms/step")

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
        log(f"cpu oracle: {out['cpu_baseline']['value']:.3e} events/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
