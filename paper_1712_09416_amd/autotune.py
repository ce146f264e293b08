"""Autotuner for the grid knobs of a batched slot.

The pad-row grid's bin size (clusters per bin aimed at, smallest bin edge)
changes how many hits each window query touches, never which hits pass the
exact window test, so the tracks do not depend on it.  For a given batch the
tuner times graph replays of every candidate, checks that each candidate's
tracks are identical to the first one's, and returns the fastest setting.
"""
from __future__ import annotations

import hashlib

import numpy as np
import torch

from .tracker import Tracker

DEFAULT_CANDIDATES = [(t, e) for t in (0.25, 0.5, 1.0) for e in (1.0, 2.0, 3.0)]


def _digest(trk: Tracker, n_events: int) -> str:
    h = hashlib.sha256()
    for e in range(n_events):
        tracks, hits = trk.get_tracks(0, e)
        h.update(tracks.tobytes())
        h.update(hits.tobytes())
    return h.hexdigest()


def autotune(geometry: dict, offsets, sector, row, y, z, candidates=None, reps: int = 5,
             **params) -> dict:
    """Time the batch (device tensors, event offsets) under each (bin_target,
    bin_min_edge) candidate.  Returns {"best": (t, e), "ms": {...}}; raises if
    any candidate's tracks differ."""
    candidates = list(candidates or DEFAULT_CANDIDATES)
    offs = np.ascontiguousarray(offsets, np.int64)
    n_events = len(offs) - 1
    total = int(offs[-1])
    ms, ref = {}, None
    for cand in candidates:
        trk = Tracker(geometry, max_events=n_events, max_clusters=total,
                      bin_target=float(cand[0]), bin_min_edge=float(cand[1]), **params)
        trk.load_batch(0, offs, sector, row, y, z)
        trk.capture(0)
        trk.launch(0)
        dig = _digest(trk, n_events)
        if ref is None:
            ref = dig
        elif dig != ref:
            trk.close()
            raise RuntimeError(f"tracks changed with grid setting {cand}")
        st = trk.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(reps):
            trk.launch(0)
        e1.record(st)
        torch.cuda.synchronize()
        ms[cand] = e0.elapsed_time(e1) / reps
        trk.close()
        del trk
    best = min(ms, key=ms.get)
    return {"best": best, "ms": ms}
