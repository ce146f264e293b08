"""Drift-velocity calibration as an asynchronous side task of the serving loop.

The paper's online calibration (Section 3, item 4) accumulates data for
every event and runs a fit every n-th event; run inline, such a task stalls
the event loop and the input buffer overflows.  Its remedy (Section 5.1):
start the long task when processing one event, check at every event whether
it has finished, and use the result as soon as it has; the result is fed
back into the cluster transformation (Section 5.3).  Here:

* accumulate: after each tracked batch, on that tracker's stream, every
  track's beam-axis z0 goes into the current histogram (library kernel);
* fit: when `every` events have been accumulated into the current
  histogram, it is closed and fitted on a stream of its own (library
  kernel, default priority) while the serving loop carries on; a fresh
  histogram takes the new events;
* feedback: the serving loop polls the fit at every iteration; when it is
  done, the library's fit has already composed the measured residual with
  the correction those events were tracked with, and the composed value
  becomes the running estimate; every later batch has its cluster z
  corrected on the device before tracking.  Histograms hold events of one
  correction only: batches are tagged with the histogram they go to, and a
  new estimate starts a new histogram.
"""
from __future__ import annotations

import torch

from .tracker import calib_fit


class _Hist:
    def __init__(self, n_bins, device, eps, stream):
        # zeroed on the side stream; trackers wait for `ready` before adding
        with torch.cuda.stream(stream):
            self.h = torch.zeros((2, n_bins), dtype=torch.int32, device=device)
            self.ready = torch.cuda.Event()
            self.ready.record(stream)
        self.eps = eps          # correction the events in it were tracked with
        self.inflight = 0       # batches submitted, not yet completed
        self.events = 0         # events completed into it
        self.closed = False


class DriftCalibration:
    def __init__(self, z_max: float, every: int = 50, n_bins: int = 4000, z_lo: float = -20.0,
                 z_hi: float = 20.0, device="cuda:0", eps0: float = 0.0):
        self.z_max, self.every = float(z_max), int(every)
        self.n_bins, self.z_lo, self.z_hi = n_bins, z_lo, z_hi
        self.device = torch.device(device)
        self.eps = float(eps0)
        self.stream = torch.cuda.Stream(self.device)
        self.out = torch.zeros(4, dtype=torch.float64, device=self.device)
        self.out_host = torch.zeros(4, dtype=torch.float64).pin_memory()
        self.cur = _Hist(n_bins, self.device, self.eps, self.stream)
        self.pending = None      # closed histogram waiting for its batches
        self.fitting = None      # (histogram, done event)
        self.history = []        # (eps measured, eps after) per fit

    # called by the server
    def on_submit(self, trk, d_sector, d_z, n: int):
        """Correct the staged clusters with the current estimate; returns
        the histogram tag of the batch."""
        if self.eps != 0.0:
            trk.calib_correct_z(d_sector[:n], d_z[:n], self.eps)
        trk.stream.wait_event(self.cur.ready)
        self.cur.h.record_stream(trk.stream)     # used there too: not reused before it is done
        self.cur.inflight += 1
        return self.cur

    def on_tracked(self, trk, tag: _Hist):
        """Accumulate the tracked batch (on its tracker's stream)."""
        trk.calib_accumulate(0, tag.h, self.z_lo, self.z_hi)

    def on_complete(self, tag: _Hist, n_events: int):
        tag.inflight -= 1
        tag.events += n_events
        if (tag is self.cur and tag.events >= self.every and self.pending is None
                and self.fitting is None):
            tag.closed = True
            self.pending = tag
            self.cur = _Hist(self.n_bins, self.device, self.eps, self.stream)

    def poll(self) -> bool:
        """Start a pending fit once all its batches are in; adopt a finished
        fit.  Never waits.  True if the estimate changed."""
        if self.pending is not None and self.pending.inflight == 0 and self.fitting is None:
            h = self.pending
            self.pending = None
            with torch.cuda.stream(self.stream):
                calib_fit(h.h, self.out, self.z_max, h.eps, self.z_lo, self.z_hi, stream=self.stream)
                self.out_host.copy_(self.out, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.stream)
            self.fitting = (h, ev)
        if self.fitting is not None and self.fitting[1].query():
            h, _ = self.fitting
            self.fitting = None
            med_a, med_c, eps_r, new = (float(v) for v in self.out_host)
            if new == new:                         # not NaN (both sides had tracks)
                self.history.append((eps_r, new))
                self.eps = new
                # events tracked with the old estimate go nowhere from now on
                self.cur = _Hist(self.n_bins, self.device, self.eps, self.stream)
                return True
        return False
