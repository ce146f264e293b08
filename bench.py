#!/usr/bin/env python3
"""Benchmark of the TPC sector tracker on one MI355X.

Workload: the central Pb-Pb-shaped event (15000 primaries + 20% secondaries
+ 5% loopers, 10% noise, 36 sectors, ~3.5M clusters), synthetic and seeded.
One step = the whole hot path over that event with its clusters already in
HBM: stage + validate, pad-row grid, neighbours finder, cleaner + start
hits, tracklet construction, ownership + selection, refit, canonical
output.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tracked clusters/s on central Pb-Pb-shaped event; p50/p99 event latency"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes of the tracklet kernel (one launch): per tracklet, the
# start hit, the seed pair and the tracklet record (64 B); per row visit,
# the hit index written, the chain link, one hit's (y, z) and the bin range
# (24 B); per hit examined in a search window, its (y, z, id) (12 B)
BYTES_PER_TRACKLET = 64
BYTES_PER_ROW_VISIT = 24
BYTES_PER_WINDOW_HIT = 12


def tracklet_bytes(cnt: dict) -> int:
    return (BYTES_PER_TRACKLET * cnt["tracklets"] + BYTES_PER_ROW_VISIT * cnt["row_visits"]
            + BYTES_PER_WINDOW_HIT * cnt["window_hits"])


def cpu_baseline(ev, threads: int) -> dict:
    """The oracle (float decisions, double refit) on the same event."""
    from oracle import oracle
    oracle.build(force=False)
    t = time.perf_counter()
    r = oracle.run_event(ev, precision=32, nthreads=threads)
    dt = time.perf_counter() - t
    return {"value": ev.n / dt, "unit": "clusters/s", "cores": threads, "kind": "oracle",
            "sample": f"whole central event ({ev.n} clusters, 36 sectors, one sector per "
                      f"thread), {dt:.2f} s, {len(r.tracks)} tracks"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="steps of the per-sector (plain) launch sequence, for comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the tracker "
              "shards by events/sectors with no exchange, see DESIGN.md", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import tpcgen
    from paper_1712_09416_amd import Tracker

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ev = tpcgen.central_event()
    print(f"bench: central event {ev.n} clusters", file=sys.stderr, flush=True)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    trk = Tracker(ev.geometry(), max_clusters=ev.n)
    torch.cuda.synchronize()

    def step():
        trk.load(0, *ins)
        trk.track_event(0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    trk.set_profiling(True)
    stage_ms = None
    counters = None
    lat = []
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_all0.record()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        ms, cnt = trk.profile()       # waits for the step
        lat.append(e0.elapsed_time(e1))
        stage_ms = {k: (stage_ms or {}).get(k, 0.0) + v for k, v in ms.items()}
        counters = cnt
    t_all1.record()
    torch.cuda.synchronize()
    total_ms = t_all0.elapsed_time(t_all1)
    trk.set_profiling(False)
    stage_ms = {k: v / args.steps for k, v in stage_ms.items()}
    tracks, hits = trk.get_tracks(0)
    ms_per_step = total_ms / args.steps
    value = ev.n / (ms_per_step * 1e-3)

    # plain: the same event with the per-sector launch sequence
    plain = None
    if args.plain_steps > 0:
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            trk.load(0, *ins)
            for s in range(36):
                trk.track_sector(0, s)
            trk.get_tracks(0)
        plain_ms = (time.perf_counter() - p0) * 1e3 / args.plain_steps
        plain = {"ms_per_event": plain_ms, "clusters_per_s": ev.n / (plain_ms * 1e-3)}

    t_tl = stage_ms["tracklets"] * 1e-3
    ach = tracklet_bytes(counters) / t_tl / 1e9
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": "k_tracklets",
            "launch_ms": stage_ms["tracklets"]}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"central Pb-Pb-shaped event, 36 sectors x 159 rows, {ev.n} clusters",
                   "mode": "fused (one launch per step over all sectors)",
                   "refit": "f64", "seed": ev.seed},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "stage_ms": stage_ms,
        "counters": counters,
        "tracks": int(len(tracks)),
        "track_hits": int(len(hits)),
        "plain": plain,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(ev, threads)
    trk.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
