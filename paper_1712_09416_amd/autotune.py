"""Autotuner for the launch shape of a batched slot.

The knobs change how the work is laid out, never what is computed: the
pad-row grid's bin size (clusters per bin aimed at, smallest bin edge)
changes how many hits each window query touches, never which hits pass the
exact window test; the tracklet kernel's block size, the window hits read
per memory round trip and the hit-list rows read per round trip by the
selection change only the order of loads and lanes.  So the tracks do not
depend on them: for a given batch the tuner times graph replays of each
candidate, checks that its tracks are identical to the first candidate's,
and keeps the fastest, one group of knobs at a time (coordinate descent).
A candidate replaces the values held so far only when it is faster by more
than a margin (1% by default, about the replays' run-to-run spread), so the
shape does not wander between equally fast ones from run to run.
"""
from __future__ import annotations

import hashlib
import itertools

import numpy as np
import torch

from .tracker import Tracker

KNOBS = {"bin_target": (0.25, 0.5, 1.0), "bin_min_edge": (1.0, 2.0, 3.0),
         "tl_block": (64, 128, 256), "win_batch": (2, 4, 8), "row_batch": (4, 8, 16)}
DEFAULTS = {"bin_target": 0.25, "bin_min_edge": 1.0, "tl_block": 64, "win_batch": 4,
            "row_batch": 8}
# groups tuned together, in this order
GROUPS = (("bin_target", "bin_min_edge"), ("tl_block",), ("win_batch",), ("row_batch",))


def _digest(trk: Tracker, n_events: int) -> str:
    h = hashlib.sha256()
    for e in range(n_events):
        tracks, hits = trk.get_tracks(0, e)
        h.update(tracks.tobytes())
        h.update(hits.tobytes())
    return h.hexdigest()


def _label(cand: dict) -> str:
    return ",".join(f"{k}={cand[k]:g}" for k in KNOBS)


def autotune(geometry: dict, offsets, sector, row, y, z, reps: int = 5, groups=GROUPS,
             knobs=None, margin: float = 0.01, **params) -> dict:
    """Tune the launch shape for the batch given as device tensors and event
    offsets.  knobs: candidate values per knob (default KNOBS); margin: the
    fraction by which a candidate must beat the values held so far.  Returns
    {"best": {knob: value}, "ms": {label: ms per replay}}; raises if any
    candidate's tracks differ from the first one's."""
    knobs = dict(KNOBS, **(knobs or {}))
    offs = np.ascontiguousarray(offsets, np.int64)
    n_events = len(offs) - 1
    total = int(offs[-1])
    ms, ref = {}, None

    def run(cand):
        nonlocal ref
        label = _label(cand)
        if label in ms:
            return ms[label]
        trk = Tracker(geometry, max_events=n_events, max_clusters=total, **cand, **params)
        try:
            trk.load_batch(0, offs, sector, row, y, z)
            trk.capture(0)
            trk.launch(0)
            dig = _digest(trk, n_events)
            if ref is None:
                ref = dig
            elif dig != ref:
                raise RuntimeError(f"tracks changed with launch shape {label}")
            st = trk.stream
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(st)
            for _ in range(reps):
                trk.launch(0)
            e1.record(st)
            torch.cuda.synchronize()
            ms[label] = e0.elapsed_time(e1) / reps
        finally:
            trk.close()
            del trk
        return ms[label]

    best = dict(DEFAULTS)
    for group in groups:
        timed = {}
        for vals in itertools.product(*(knobs[k] for k in group)):
            cand = dict(best)
            cand.update(zip(group, vals))
            timed[vals] = run(cand)
        held = tuple(best[k] for k in group)
        top = min(timed, key=timed.get)
        if held not in timed or timed[top] < timed[held] * (1.0 - margin):
            best.update(zip(group, top))
    return {"best": best, "ms": ms, "best_ms": ms[_label(best)]}
