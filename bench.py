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

# Algorithmic bytes (what the method has to move, counted per unit of work
# with the units counted on the device in the same run):
#  - the tracklet kernel, per launch: 20 B per tracklet row visit (the hit's
#    y/z, its chain link and the row's bin range) + 14 B per tracklet hit
#    (the hit-list entry and the ownership weight's read-modify-write);
#  - the whole path, per event: 67 B per cluster (grid 30, neighbours 24,
#    cleaner + start hits 13) + the tracklet terms + 12 B per track hit
#    (list, weight, y/z read, ID written) + 84 B per output track.
BYTES_PER_ROW_VISIT = 20
BYTES_PER_TRACKLET_HIT = 14
BYTES_PER_CLUSTER = 67
BYTES_PER_TRACK_HIT = 12
BYTES_PER_TRACK = 84

# VALU issue peak: 256 CUs x 4 SIMDs, each issuing one wave64 vector
# instruction per 4 cycles at 2.4 GHz
VALU_PEAK_GINST_S = 256 * 4 * 2.4 / 4.0

# Counter summaries of the tracklet kernel (rocprofv3 --pmc runs), used only
# while the kernel's sources are those the counters were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tracklets_central_pbpb_traffic.md")
SQ_FILE = os.path.join(ROOT, "profiles", "k_tracklets_central_pbpb_sq.md")
KERNEL_SOURCES = ("paper_1712_09416_amd/csrc/tracklet.hip", "paper_1712_09416_amd/csrc/tpc_device.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _summary_value(path: str, key: str):
    """Integer `key: value` of a committed counter summary, or None if the
    file is absent or was taken on other kernel sources."""
    import re
    try:
        txt = open(path).read()
    except OSError:
        return None
    m = re.search(key + r":\s*([0-9]+)", txt)
    hsh = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    if not m or not hsh or hsh.group(1) != kernel_source_hash():
        return None
    return int(m.group(1))


def measured_traffic():
    """L2-miss bytes (FETCH_SIZE + WRITE_SIZE, scaled) per tracklet launch."""
    return _summary_value(TRAFFIC_FILE, "traffic_bytes_per_launch")


def measured_valu():
    """VALU wave instructions (SQ_INSTS_VALU) per tracklet launch."""
    return _summary_value(SQ_FILE, "valu_insts_per_launch")


def tracklet_bytes(cnt: dict) -> int:
    return BYTES_PER_ROW_VISIT * cnt["row_visits"] + BYTES_PER_TRACKLET_HIT * cnt["tracklet_hits"]


def path_bytes(cnt: dict) -> int:
    return (BYTES_PER_CLUSTER * cnt["clusters"] + tracklet_bytes(cnt)
            + BYTES_PER_TRACK_HIT * cnt["track_hits"] + BYTES_PER_TRACK * cnt["tracks"])


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def host_threads() -> int:
    """CPU threads this process may use (its affinity), at most 16 (the
    share of one GPU's host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class Ev:
    """Cluster arrays of a generated event (from tpcgen.parallel)."""

    def __init__(self, d):
        self.sector, self.row, self.y, self.z = d["sector"], d["row"], d["y"], d["z"]
        self.sigma = d["sigma"]
        self.name = d["name"]
        self.n = int(len(self.y))
        self.seed = None

    def geometry(self):
        from tpcgen import geometry as G
        return G.geometry_dict(self.sigma)


def serve_pool_specs():
    """Distinct events the serving stream draws from: pp-like, peripheral
    (2000 primaries, Pb-Pb shape) and central."""
    import tpcgen
    specs = [("pp", (tpcgen.seed_for(4, e),)) for e in range(24)]
    specs += [("pbpb", (tpcgen.seed_for(4, 100 + e), 2000)) for e in range(8)]
    specs += [("pbpb", (tpcgen.seed_for(4, 200 + e), 15000)) for e in range(2)]
    return specs


def bench_batch(evs, geo, dev, steps: int) -> dict:
    """64 events of uneven size (Pb-Pb shape, multiplicity log-uniform
    50-15000): tracked together in one slot (one launch per step over all
    2304 sectors), replayed from a HIP graph, with the grid knobs autotuned
    on the batch; the same events over 2-4 slots replayed in flight on their
    own streams; compared with the one slot without the graph, with one
    event at a time (fused launches) and with the plain per-sector launch
    sequence."""
    import numpy as np
    import torch
    from paper_1712_09416_amd import Tracker
    evs = [Ev(d) for d in evs]
    offs = np.concatenate([[0], np.cumsum([e.n for e in evs])]).astype(np.int64)
    total = int(offs[-1])
    cat = [torch.from_numpy(np.concatenate([getattr(e, k) for e in evs])).to(dev)
           for k in ("sector", "row", "y", "z")]
    # launch shape tuned on this batch (the tuner checks the tracks do not change)
    from paper_1712_09416_amd.autotune import autotune
    tune = autotune(geo, offs, *cat, reps=3)
    print(f"bench: batch autotune {tune}", file=sys.stderr, flush=True)
    trk = Tracker(geo, max_events=len(evs), max_clusters=total, **tune["best"])
    st = trk.stream

    def timed(fn, reps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    trk.load_batch(0, offs, *cat)
    trk.track_event(0)
    ntracks = sum(len(trk.get_tracks(0, e)[0]) for e in range(len(evs)))
    trk.load_batch(0, offs, *cat)
    trk.capture(0)
    trk.launch(0)
    ms_graph = timed(lambda: trk.launch(0), steps)

    # the same 64 events over k slots in flight: k trackers (streams), each
    # replaying the graph of its share of the events (largest first, dealt
    # round-robin), so one slot's latency-bound tails overlap the others'
    # work; the host clock around the synchronised replays
    sizes = offs[1:] - offs[:-1]
    order = np.argsort(-sizes, kind="stable")
    inflight = {}
    for k in (2, 3, 4):
        pool = []
        for j in range(k):
            idx = np.sort(order[j::k])
            sub_off = np.concatenate([[0], np.cumsum(sizes[idx])]).astype(np.int64)
            sub = [torch.cat([c[offs[i]:offs[i + 1]] for i in idx]) for c in cat]
            t = Tracker(geo, max_events=len(idx), max_clusters=max(1, int(sub_off[-1])),
                        **tune["best"])
            t.load_batch(0, sub_off, *sub)
            t.capture(0)
            t.launch(0)
            pool.append((t, sub))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for t, _sub in pool:
                t.launch(0)
        torch.cuda.synchronize()
        inflight[k] = (time.perf_counter() - t0) * 1e3 / steps
        nt_k = sum(len(t.get_tracks(0, e)[0]) for t, sub in pool
                   for e in range(t.params.max_events))
        assert nt_k == ntracks, ("slots in flight disagree with the one slot", nt_k, ntracks)
        for t, _sub in pool:
            t.close()
        del pool
    k_best = min(inflight, key=inflight.get)

    def eager():
        trk.load_batch(0, offs, *cat)
        trk.track_event(0)
    eager()
    ms_eager = timed(eager, steps)
    slices = [[c[offs[e]:offs[e + 1]] for c in cat] for e in range(len(evs))]

    def per_event():
        for sl in slices:
            trk.load(0, *sl)
            trk.track_event(0)
    per_event()
    ms_events = timed(per_event, 1)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for sl in slices:
        trk.load(0, *sl)
        for s in range(36):
            trk.track_sector(0, s)
        trk.device_results(0)
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - p0) * 1e3
    trk.close()
    rate = lambda ms: total / (ms * 1e-3)  # noqa: E731
    return {"events": len(evs), "clusters": total, "sectors": 36 * len(evs), "tracks": ntracks,
            "graph_ms": ms_graph, "graph_clusters_per_s": rate(ms_graph),
            "graph_slots_in_flight": {"best_slots": k_best, "ms": inflight[k_best],
                                      "clusters_per_s": rate(inflight[k_best]),
                                      "ms_by_slots": inflight},
            "one_launch_per_step_ms": ms_eager, "one_launch_per_step_clusters_per_s": rate(ms_eager),
            "per_event_ms": ms_events, "per_event_clusters_per_s": rate(ms_events),
            "plain_ms": ms_plain, "plain_clusters_per_s": rate(ms_plain),
            "autotune": {"best": tune["best"], "graph_ms": tune["ms"]}}


def bench_serve(pool, geo, n_req: int) -> dict:
    """Poisson stream of events (70% pp, 25% peripheral, 5% central, drawn
    from a pool of distinct events), served with continuous batching over 4
    streams vs the plain one-event-at-a-time path.  Rates: 0.7 x the plain
    capacity (both modes), and 0.7 x the continuous-batching capacity."""
    import numpy as np
    from paper_1712_09416_amd.serve import Server, Request, poisson_arrivals
    evs = [Ev(d) for d in pool]
    kinds = {"pp": [e for e in evs if e.name.startswith("pp")],
             "peripheral": [e for e in evs if e.name == "pbpb_2000"],
             "central": [e for e in evs if e.name == "pbpb_15000"]}
    rng = np.random.default_rng(1712094164)
    warm = max(30, n_req // 10)
    u = rng.uniform(size=n_req + warm)
    kind = np.where(u < 0.70, "pp", np.where(u < 0.95, "peripheral", "central"))
    picks = []
    counters = {k: 0 for k in kinds}
    for k in kind:
        picks.append(kinds[k][counters[k] % len(kinds[k])])
        counters[k] += 1
    cap = max(e.n for e in evs) + 1024
    # launch shape tuned on a continuous-batching slot of the mix: the first
    # 8 requests of the stream in one slot
    import torch
    from paper_1712_09416_amd.autotune import autotune
    slot = picks[:8]
    offs = np.concatenate([[0], np.cumsum([e.n for e in slot])]).astype(np.int64)
    cat = [torch.from_numpy(np.concatenate([getattr(e, k) for e in slot])).cuda()
           for k in ("sector", "row", "y", "z")]
    tune = autotune(geo, offs, *cat, reps=5)
    shape = tune["best"]
    del cat
    print(f"bench: serving-mix autotune {tune}", file=sys.stderr, flush=True)

    # events of 100k clusters or more arrive in pinned host memory (as from
    # a DMA engine) and go to the device from there; the small ones arrive in
    # numpy arrays and are staged through each tracker's pinned buffers
    src = {}
    for e in evs:
        arrs = (e.sector, e.row, e.y, e.z)
        src[id(e)] = ([torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in arrs]
                      if e.n >= 100_000 else arrs)

    def requests(times):
        return [Request(float(t), *src[id(e)], tag=e.name) for t, e in zip(times, picks)]

    def capacity(plain):
        srv = Server(geo, n_streams=4, max_events=32, cap_clusters=cap, plain=plain, **shape)
        srv.run(requests(np.zeros(len(picks[:40])))[:40])          # warm-up
        st = srv.run(requests(np.zeros(len(picks))))
        srv.close()
        return st.n_requests / st.wall_s

    def serve(plain, rate):
        srv = Server(geo, n_streams=4, max_events=32, cap_clusters=cap, plain=plain, **shape)
        srv.run(requests(np.zeros(40))[:40])
        st = srv.run(requests(poisson_arrivals(len(picks), rate, seed=7)), warmup=warm)
        srv.close()
        out = st.summary()
        print(f"bench: serve plain={plain} rate {rate:.1f}/s: {out}", file=sys.stderr, flush=True)
        return out

    def serve_calib(rate, with_calib):
        """The same stream with a 0.4% drift-velocity error in every event,
        with or without the calibration side task."""
        import tpcgen
        from paper_1712_09416_amd.calib import DriftCalibration
        dist = {id(e): tpcgen.drift_z(e.sector, e.z, 0.004) for e in picks}
        times = poisson_arrivals(len(picks), rate, seed=7)
        rq = [Request(float(t), e.sector, e.row, e.y, dist[id(e)], tag=e.name)
              for t, e in zip(times, picks)]
        cal = DriftCalibration(250.0, every=50) if with_calib else None
        srv = Server(geo, n_streams=4, max_events=32, cap_clusters=cap, calib=cal, **shape)
        srv.run(rq[:40])
        st = srv.run(rq, warmup=warm)
        srv.close()
        out = st.summary()
        if cal is not None:
            out["calibration"] = {"fits": len(cal.history), "eps_true": 0.004, "eps_final": cal.eps,
                                  "every_events": 50}
        print(f"bench: serve drift calib={with_calib} rate {rate:.1f}/s: {out}", file=sys.stderr,
              flush=True)
        return out

    def calib_ab(rate, reps=3):
        """Without / with the side task, alternated (run-to-run spread of the
        latencies is larger than the side task's cost); medians."""
        runs = {False: [], True: []}
        for _ in range(reps):
            for w in (False, True):
                runs[w].append(serve_calib(rate, w))
        med = lambda rs, k: float(np.median([r[k] for r in rs]))  # noqa: E731
        out = {"rate_events_per_s": rate, "repeats": reps}
        for w, name in ((False, "without"), (True, "with")):
            out[name] = {"p50_ms": med(runs[w], "p50_ms"), "p99_ms": med(runs[w], "p99_ms"),
                         "runs": [{"p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"]} for r in runs[w]]}
        out["with"]["calibration"] = runs[True][-1]["calibration"]
        return out

    c_plain = capacity(True)
    print(f"bench: serve plain capacity {c_plain:.1f} events/s", file=sys.stderr, flush=True)
    c_cb = capacity(False)
    print(f"bench: serve batching capacity {c_cb:.1f} events/s", file=sys.stderr, flush=True)
    r1 = 0.7 * c_plain
    return {"mix": "70% pp / 25% peripheral (2000 primaries) / 5% central, pool of 34 distinct events",
            "autotune": {"slot": "first 8 requests of the stream", "best": shape, "graph_ms": tune["ms"]},
            "capacity_events_per_s": {"plain": c_plain, "continuous_batching": c_cb},
            "at_0.7_plain_capacity": {"rate_events_per_s": r1, "plain": serve(True, r1),
                                      "continuous_batching": serve(False, r1)},
            "at_0.7_cb_capacity": {"rate_events_per_s": 0.7 * c_cb,
                                   "continuous_batching": serve(False, 0.7 * c_cb)},
            "drift_calibration_side_task": calib_ab(0.7 * c_cb)}


def cpu_baseline(ev, threads: int, reps: int = 3, sample_sectors: int = 6) -> dict:
    """The oracle (float decisions, double refit; as it stands, one sector
    per thread) timed on the host: the whole central event on `threads`
    threads, and a sample of its first `sample_sectors` sectors (their
    clusters only; sectors are tracked independently) on one thread; median
    of `reps` runs each."""
    import numpy as np
    from oracle import oracle
    oracle.build(force=False)
    geo = ev.geometry()

    def timed(sel, nthreads):
        ts, nt = [], 0
        for _ in range(reps):
            t = time.perf_counter()
            r = oracle.run(ev.sector[sel], ev.row[sel], ev.y[sel], ev.z[sel], geo, precision=32,
                           nthreads=nthreads)
            ts.append(time.perf_counter() - t)
            nt = len(r.tracks)
        return float(np.median(ts)), ts, nt

    everything = slice(None)
    dt, ts, nt = timed(everything, threads)
    sel = np.nonzero(ev.sector < sample_sectors)[0]
    dt1, ts1, nt1 = timed(sel, 1)
    model = cpu_model()
    return {"value": ev.n / dt, "unit": "clusters/s", "cores": threads, "kind": "oracle",
            "cpu_model": model,
            "sample": f"whole central event ({ev.n} clusters, 36 sectors, one sector per thread), "
                      f"median of {reps} runs: {dt:.2f} s, {nt} tracks",
            "runs_s": ts,
            "single_thread": {"value": len(sel) / dt1, "unit": "clusters/s", "cores": 1,
                              "sample": f"sectors 0-{sample_sectors - 1} of the central event "
                                        f"({len(sel)} clusters), median of {reps} runs: "
                                        f"{dt1:.2f} s, {nt1} tracks",
                              "runs_s": ts1}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--central-shape", default="",
                    help="launch shape of the central event as k=v,... (skips its autotuning)")
    ap.add_argument("--no-single-stream", action="store_true",
                    help="skip the one-event-at-a-time reference run (counter runs)")
    ap.add_argument("--inflight", type=int, default=3,
                    help="events in flight (one tracker context and stream each)")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="steps of the per-sector (plain) launch sequence, for comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for counter scaling)")
    ap.add_argument("--merge-reps", type=int, default=5,
                    help="timed runs of the cross-sector merger on the central event (0: skip)")
    ap.add_argument("--e2e-steps", type=int, default=20,
                    help="end-to-end steps (host clusters in, host tracks out)")
    ap.add_argument("--batch-events", type=int, default=64,
                    help="events of the batched workload (0: skip it)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving workload (0: skip it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for {args.gpus}); events and sectors are "
              "independent, so more GPUs would each take whole events", file=sys.stderr)
        return 2

    import numpy as np
    import tpcgen
    from tpcgen import parallel

    # every synthetic event is generated before the GPU is touched
    mult = tpcgen.batch_multiplicities(64)[: args.batch_events]
    specs = [("central", ())]
    specs += [("batch", (e, int(m))) for e, m in enumerate(mult)]
    serve_specs = serve_pool_specs() if args.serve_requests > 0 else []
    gen = parallel.generate(specs + serve_specs)
    central = gen[0]
    batch_evs = gen[1:1 + len(mult)]
    serve_pool = gen[1 + len(mult):]

    import torch
    from paper_1712_09416_amd import Tracker

    dev = torch.device("cuda:0")
    # a plain 1 GiB device copy: the practical bandwidth ceiling on this GPU,
    # and the reference kernel for scaling the HBM byte counters
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_copy = 1 if args.copy_calibration else 10
    torch.cuda.synchronize()
    c0.record()
    for _ in range(n_copy):
        b.copy_(a)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * a.numel() * n_copy / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del a, b
    ev = Ev(central)
    print(f"bench: central event {ev.n} clusters", file=sys.stderr, flush=True)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    # the launch shape tuned on this event (graph replays; the tuner checks
    # that the tracks do not change)
    from paper_1712_09416_amd.autotune import autotune, DEFAULTS
    if args.central_shape:
        # a given shape (e.g. for counter runs): no tuning
        shape = dict(DEFAULTS)
        for kv in args.central_shape.split(","):
            k, v = kv.split("=")
            shape[k] = type(DEFAULTS[k])(float(v))
        tune_c = {"best": shape, "ms": {}, "given": True}
    else:
        tune_c = autotune(ev.geometry(), np.array([0, ev.n], np.int64), *ins, reps=5)
    print(f"bench: central autotune {tune_c}", file=sys.stderr, flush=True)
    # events in flight: one tracker context per stream, step i on tracker
    # i mod n (each event's whole path on its tracker's stream; the events
    # of different streams overlap on the GPU, the paper's pipelined events)
    n_fl = max(1, args.inflight)
    trks = [Tracker(ev.geometry(), max_clusters=ev.n, **tune_c["best"]) for _ in range(n_fl)]
    trk = trks[0]
    st = trk.stream
    torch.cuda.synchronize()

    def run_steps(pool, k_steps, merge=False):
        """k_steps steps, step i on pool[i % len(pool)], with the library's
        stage events on (HIP events between the stages on each tracker's
        stream, no synchronisation); with merge, each step also runs the
        cross-sector merger on its event.  Returns the host wall time, the
        per-step HIP-event latencies, the per-stage means over these steps
        (averaged over the trackers) and the work counters."""
        for t in pool:
            t.set_profiling(True)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(k_steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i, (e0, e1) in enumerate(evs):
            t = pool[i % len(pool)]
            e0.record(t.stream)
            t.load(0, *ins)
            t.track_event(0)
            if merge:
                t.merge(0)
            e1.record(t.stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) * 1e3
        lats = [e0.elapsed_time(e1) for e0, e1 in evs]
        prof = [t.profile() for t in pool[:min(len(pool), k_steps)]]
        for t in pool:
            t.set_profiling(False)
        stages = {k: float(np.mean([p[0][k] for p in prof])) for k in prof[0][0]}
        return wall, lats, stages, prof[0][1]

    for i in range(args.warmup):
        trks[i % n_fl].load(0, *ins)
        trks[i % n_fl].track_event(0)
    torch.cuda.synchronize()

    # timed region: K steps, n_fl events in flight
    wall_ms, lat, stage_ms, counters = run_steps(trks, args.steps)
    # the same K steps on one stream (one event at a time), for reference
    if args.no_single_stream:
        wall1_ms, lat1, stage1_ms = wall_ms, lat, stage_ms
    else:
        wall1_ms, lat1, stage1_ms, _ = run_steps(trks[:1], args.steps)

    # end to end: clusters in pinned host memory -> tracks in (pinned) host
    # memory
    e2e = []
    if args.e2e_steps > 0:
        from paper_1712_09416_amd._lib import TRACK_DTYPE
        pin = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
               for a in (ev.sector, ev.row, ev.y, ev.z)]
        p = trk.params
        max_tracks = p.max_clusters // p.n_min_track + 36
        out_t = torch.empty(max_tracks * TRACK_DTYPE.itemsize, dtype=torch.uint8,
                            pin_memory=True).numpy().view(TRACK_DTYPE)
        out_h = torch.empty(ev.n, dtype=torch.int32, pin_memory=True).numpy()
        for k in range(args.e2e_steps + 2):
            t0 = time.perf_counter()
            trk.load(0, *pin)
            trk.track_event(0)
            trk.get_slot_tracks(0, out_t, out_h)
            if k >= 2:
                e2e.append((time.perf_counter() - t0) * 1e3)

    # tracking and merging each event, the same events in flight: the
    # merger's latency-bound kernels share the GPU with the other events'
    merge_inflight = None
    if args.merge_reps > 0 and args.steps > 0:
        wall_m, lat_m, _, _ = run_steps(trks, args.steps, merge=True)
        merge_inflight = {"ms_per_step": wall_m / args.steps,
                          "clusters_per_s": ev.n / (wall_m / args.steps * 1e-3),
                          "p50_ms": float(np.percentile(lat_m, 50)),
                          "events_in_flight": n_fl}

    tracks, hits = trk.get_tracks(0)
    # the trackers of the pipeline that tracked the event (fewer than
    # n_fl when the run has fewer steps)
    n_ran = min(n_fl, max(args.steps, args.warmup))
    for i, t in enumerate(trks[1:], start=1):
        if i < n_ran:
            th, hh = t.get_tracks(0)
            assert np.array_equal(hh, hits) and np.array_equal(th["par"], tracks["par"]), \
                "trackers of the pipelined run disagree"
        t.close()
    # whole-job rate from the host clock around the synchronised region
    ms_per_step = wall_ms / args.steps
    value = ev.n / (ms_per_step * 1e-3)
    single_stream = {"ms_per_step": wall1_ms / args.steps,
                     "clusters_per_s": ev.n / (wall1_ms / args.steps * 1e-3),
                     "p50_ms": float(np.percentile(lat1, 50)),
                     "p99_ms": float(np.percentile(lat1, 99)), "stage_ms": stage1_ms}

    # cross-sector merger on the tracked central event (the step after the
    # per-sector path; timed on its own, not part of the step above)
    merge = None
    if args.merge_reps > 0:
        trk.load(0, *ins)
        trk.track_event(0)
        trk.merge(0)
        torch.cuda.synchronize()
        m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        m0.record(st)
        for _ in range(args.merge_reps):
            trk.merge(0)
        m1.record(st)
        torch.cuda.synchronize()
        mt, mh, mseg = trk.get_merged(0)
        merge = {"ms": m0.elapsed_time(m1) / args.merge_reps, "tracks_in": int(len(tracks)),
                 "tracks_out": int(len(mt)), "chains": int((mseg > 1).sum()),
                 "track_and_merge_in_flight": merge_inflight}

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
        # the same per-sector sequences spread over 4 streams (concurrent sectors)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            trk.load(0, *ins)
            trk.track_event_streams(0, 4)
            trk.get_tracks(0)
        ms4 = (time.perf_counter() - p0) * 1e3 / args.plain_steps
        plain["streams4_ms_per_event"] = ms4
        plain["streams4_clusters_per_s"] = ev.n / (ms4 * 1e-3)

    # roofline of the dominant kernel (k_tracklets, one launch per step):
    # algorithmic bytes 20 V + 14 H_t over its mean launch time in the timed
    # region; the limiter named from its counters (VALU issue share against
    # the L2-miss traffic's share of the HBM peak)
    t_tl = stage_ms["tracklets"] * 1e-3
    ach = tracklet_bytes(counters) / t_tl / 1e9
    traffic = measured_traffic()
    valu = measured_valu()
    shares = {}
    if traffic is not None:
        shares["hbm"] = traffic / t_tl / 1e9 / HBM_PEAK_GBS
    if valu is not None:
        shares["alu"] = valu / t_tl / 1e9 / VALU_PEAK_GINST_S
    # no counters for these kernel sources: the limiter is not named
    bound = max(shares, key=shares.get) if shares else None
    roof = {"bound": bound, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_tracklets",
            "algorithmic_bytes": tracklet_bytes(counters),
            "bytes_formula": "20 x row visits + 14 x tracklet hits",
            "launch_ms": stage_ms["tracklets"], "copy_kernel_gbs": copy_gbs,
            "limiter_shares": shares,
            "limiter_note": ("VALU issue share vs L2-miss traffic share of the HBM peak, from "
                             "the committed counters" if shares else
                             "counters were taken on other kernel sources: limiter unmeasured"),
            "traffic_note": "traffic = L2-miss bytes (FETCH_SIZE + WRITE_SIZE, scaled by a "
                            "copy kernel), most of it served by the Infinity Cache"}
    if traffic is not None:
        roof["traffic_gbs"] = traffic / t_tl / 1e9
    if valu is not None:
        roof["alu"] = {"valu_insts_per_launch": valu, "achieved_ginst_s": valu / t_tl / 1e9,
                       "peak_ginst_s": VALU_PEAK_GINST_S,
                       "frac": valu / t_tl / 1e9 / VALU_PEAK_GINST_S}
    # the same kernel when one event runs alone on the GPU
    t_tl1 = stage1_ms["tracklets"] * 1e-3
    roof["single_stream"] = {"launch_ms": stage1_ms["tracklets"],
                             "achieved": tracklet_bytes(counters) / t_tl1 / 1e9,
                             "frac": tracklet_bytes(counters) / t_tl1 / 1e9 / HBM_PEAK_GBS}
    # the whole path per step: 67 N + 20 V + 14 H_t + 12 H_k + 84 K
    pb = path_bytes(counters)
    roof["whole_path"] = {"algorithmic_bytes": pb,
                          "bytes_formula": "67 N + 20 V + 14 H_t + 12 H_k + 84 K",
                          "achieved": pb / (ms_per_step * 1e-3) / 1e9,
                          "frac": pb / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS}

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
                   "events_in_flight": n_fl,
                   "launch_shape": tune_c["best"],
                   "refit": "f64", "seed": tpcgen.seed_for(2)},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "latency_note": "per-event HIP-event time on its tracker's stream, with the other "
                        "events in flight sharing the GPU",
        "stage_ms": stage_ms,
        "single_stream": single_stream,
        "counters": counters,
        "tracks": int(len(tracks)),
        "track_hits": int(len(hits)),
        "plain": plain,
        "merge": merge,
        "end_to_end": ({"what": "pinned host clusters -> H2D -> tracking -> tracks in pinned host memory",
                        "p50_ms": float(np.percentile(e2e, 50)),
                        "p99_ms": float(np.percentile(e2e, 99)),
                        "clusters_per_s": ev.n / (float(np.mean(e2e)) * 1e-3)} if e2e else None),
        "roofline": roof,
        "autotune": {"central": {"best": tune_c["best"], "graph_ms": tune_c["ms"]}},
    }
    trk.close()
    print(f"bench: central {ms_per_step:.3f} ms/step, stages {stage_ms}", file=sys.stderr, flush=True)
    if len(batch_evs):
        out["batch"] = bench_batch(batch_evs, ev.geometry(), dev, args.batch_steps)
        print(f"bench: batch {out['batch']}", file=sys.stderr, flush=True)
    if args.serve_requests > 0:
        out["serve"] = bench_serve(serve_pool, ev.geometry(), args.serve_requests)
        print(f"bench: serve {out['serve']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ev, host_threads())
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
