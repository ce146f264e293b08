"""Serving loop: events arrive over time and are tracked as they come.

The online setting of the paper's tracker (Section 2: the HLT processes a
continuous stream of events, many in flight at once, pipelined through the
chain).  Here, on one GPU:

* requests (events in host memory) arrive with given arrival times;
* a request is admitted when one of the trackers (one per HIP stream) is
  free and the clusters in flight stay within a device cluster budget;
* a freed tracker takes every waiting request that fits (continuous
  batching: the events share one slot and one launch per step), copies them
  through pinned host memory to the device and enqueues the tracking, all on
  its own stream, so the copies and kernels of different trackers overlap;
* a request completes when its tracks are back in host memory; latency =
  completion - arrival.

Mode "plain" is the reference: one tracker, one event at a time, tracked
with the per-sector launch sequence.

With `calib` (a DriftCalibration), a drift-velocity calibration runs beside
the loop: every batch's clusters get the current z correction before
tracking and its tracks are accumulated; fits run on a stream of their own
and are polled, never waited for (paper, Sections 3 and 5.1).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from .tracker import TRACK_DTYPE, Tracker


@dataclass
class Request:
    """One event: its clusters in host memory, as numpy arrays or as pinned
    CPU tensors (as a DMA engine would deliver them), which are transferred
    to the device without a host copy."""
    arrival: float                 # seconds from the start of the run
    sector: np.ndarray
    row: np.ndarray
    y: np.ndarray
    z: np.ndarray
    tag: str = ""

    @property
    def n(self) -> int:
        return int(self.y.shape[0])


@dataclass
class ServeStats:
    mode: str
    n_requests: int
    clusters: int
    wall_s: float
    latency_ms: np.ndarray
    results: list = field(default_factory=list)

    def summary(self) -> dict:
        lat = self.latency_ms
        return {"mode": self.mode, "requests": self.n_requests, "clusters": self.clusters,
                "wall_s": self.wall_s, "clusters_per_s": self.clusters / self.wall_s,
                "events_per_s": self.n_requests / self.wall_s,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean())}


class _Worker:
    """One tracker on its own stream with pinned staging buffers."""

    def __init__(self, geometry, max_events, cap, device, **params):
        self.trk = Tracker(geometry, max_events=max_events, max_clusters=cap, device=device,
                           **params)
        self.cap = cap
        pin = dict(pin_memory=True)
        self.h_sector = torch.empty(cap, dtype=torch.uint8, **pin)
        self.h_row = torch.empty(cap, dtype=torch.uint8, **pin)
        self.h_y = torch.empty(cap, dtype=torch.float32, **pin)
        self.h_z = torch.empty(cap, dtype=torch.float32, **pin)
        self.d_sector = torch.empty(cap, dtype=torch.uint8, device=device)
        self.d_row = torch.empty(cap, dtype=torch.uint8, device=device)
        self.d_y = torch.empty(cap, dtype=torch.float32, device=device)
        self.d_z = torch.empty(cap, dtype=torch.float32, device=device)
        # pinned result buffers for the slot's most tracks and hits: the
        # results come back into them (much faster than into pageable memory)
        p = self.trk.params
        max_tracks = p.max_clusters // p.n_min_track + 36 * max_events
        self.r_tracks_t = torch.empty(max_tracks * TRACK_DTYPE.itemsize, dtype=torch.uint8, **pin)
        self.r_tracks = self.r_tracks_t.numpy().view(TRACK_DTYPE)
        self.r_hits_t = torch.empty(cap, dtype=torch.int32, **pin)
        self.r_hits = self.r_hits_t.numpy()
        self.batch: list[int] = []

    def submit(self, reqs: list[Request], ids: list[int], plain: bool, calib=None):
        # requests in host numpy arrays are staged through the pinned buffers
        # (one host copy each, then one transfer per field for all of them);
        # requests already in pinned host tensors are transferred from where
        # they are, after the staged ones
        staged = [i for i in ids if not isinstance(reqs[i].y, torch.Tensor)]
        direct = [i for i in ids if isinstance(reqs[i].y, torch.Tensor)]
        ids = staged + direct
        offs = np.zeros(len(ids) + 1, np.int64)
        for k, i in enumerate(ids):
            offs[k + 1] = offs[k] + reqs[i].n
        n = int(offs[-1])
        ns = int(offs[len(staged)])
        hs, hr, hy, hz = (t.numpy() for t in (self.h_sector, self.h_row, self.h_y, self.h_z))
        for k, i in enumerate(staged):
            a, b = offs[k], offs[k + 1]
            r = reqs[i]
            hs[a:b] = r.sector
            hr[a:b] = r.row
            hy[a:b] = r.y
            hz[a:b] = r.z
        dev = (self.d_sector, self.d_row, self.d_y, self.d_z)
        with torch.cuda.stream(self.trk.stream):
            if ns:
                for d, h in zip(dev, (self.h_sector, self.h_row, self.h_y, self.h_z)):
                    d[:ns].copy_(h[:ns], non_blocking=True)
            for k, i in enumerate(direct, start=len(staged)):
                a, b = int(offs[k]), int(offs[k + 1])
                r = reqs[i]
                for d, src in zip(dev, (r.sector, r.row, r.y, r.z)):
                    d[a:b].copy_(src, non_blocking=True)
            self.tag = calib.on_submit(self.trk, self.d_sector, self.d_z, n) if calib else None
            self.trk.load_batch(0, offs, self.d_sector[:n], self.d_row[:n], self.d_y[:n],
                                self.d_z[:n])
        if plain:
            for s in range(36 * len(ids)):
                self.trk.track_sector(0, s)
        else:
            self.trk.submit(0)
        if calib:
            # on the tracker's stream: the histogram's zeroing is already
            # ordered by on_submit, and nothing else needs torch's stream
            with torch.cuda.stream(self.trk.stream):
                calib.on_tracked(self.trk, self.tag)
        self.batch = list(ids)

    def close(self):
        self.trk.close()


class Server:
    """n_streams trackers; each slot holds up to max_events events and
    cap_clusters clusters; at most budget_clusters clusters in flight;
    params: tracker params (e.g. a tuned launch shape)."""

    def __init__(self, geometry: dict, n_streams: int = 4, max_events: int = 32,
                 cap_clusters: int = 4 << 20, budget_clusters: int | None = None,
                 device: str = "cuda:0", plain: bool = False, calib=None, **params):
        self.plain = plain
        self.calib = calib        # optional DriftCalibration side task
        if plain:
            n_streams, max_events = 1, 1
        self.max_events = max_events
        self.workers = [_Worker(geometry, max_events, cap_clusters, device, **params)
                        for _ in range(n_streams)]
        self.cap = cap_clusters
        self.budget = budget_clusters if budget_clusters is not None else n_streams * cap_clusters

    def run(self, reqs: list[Request], collect: bool = False, warmup: int = 0) -> ServeStats:
        """Serve the requests (sorted by arrival).  The first `warmup`
        requests are served but left out of the statistics."""
        for r in reqs:
            if r.n > self.cap or r.n > self.budget:
                raise ValueError(f"request with {r.n} clusters exceeds the slot capacity")
        order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival)
        pending = deque()
        done_at = np.zeros(len(reqs))
        results = [None] * len(reqs) if collect else []
        free = list(range(len(self.workers)))
        busy = {}
        in_flight = 0
        nxt = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while nxt < len(order) or pending or busy:
            now = time.perf_counter() - t0
            while nxt < len(order) and reqs[order[nxt]].arrival <= now:
                pending.append(order[nxt])
                nxt += 1
            progressed = False
            if self.calib and self.calib.poll():      # side task: never waits
                progressed = True
            # completions
            for w in list(busy):
                wk = self.workers[w]
                if not wk.trk.poll(0):
                    continue
                out = wk.trk.get_slot_tracks(0, wk.r_tracks, wk.r_hits)
                for e, i in enumerate(wk.batch):
                    tracks, hits = out[e]
                    done_at[i] = time.perf_counter() - t0
                    in_flight -= reqs[i].n
                    if collect:      # the worker's buffers are reused: keep copies
                        results[i] = (tracks.copy(), hits.copy())
                if self.calib:
                    self.calib.on_complete(wk.tag, len(wk.batch))
                del busy[w]
                free.append(w)
                progressed = True
            # admission: a free tracker takes every waiting request that fits
            while free and pending:
                take, n = [], 0
                while (pending and len(take) < self.max_events
                       and n + reqs[pending[0]].n <= self.cap
                       and in_flight + n + reqs[pending[0]].n <= self.budget):
                    i = pending.popleft()
                    take.append(i)
                    n += reqs[i].n
                if not take:
                    break
                w = free.pop()
                self.workers[w].submit(reqs, take, self.plain, self.calib)
                busy[w] = True
                in_flight += n
                progressed = True
            if not progressed:
                if busy:
                    time.sleep(20e-6)
                elif nxt < len(order):
                    time.sleep(max(0.0, min(1e-3, reqs[order[nxt]].arrival - now)))
        wall = time.perf_counter() - t0
        keep = order[warmup:]
        lat = np.array([(done_at[i] - reqs[i].arrival) * 1e3 for i in keep])
        first = min(reqs[i].arrival for i in keep)
        span = max(done_at[i] for i in keep) - first
        return ServeStats(mode="plain" if self.plain else "continuous-batching",
                          n_requests=len(keep), clusters=int(sum(reqs[i].n for i in keep)),
                          wall_s=span if span > 0 else wall, latency_ms=lat, results=results)

    def close(self):
        for w in self.workers:
            w.close()


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
