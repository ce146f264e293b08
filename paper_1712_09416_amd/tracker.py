"""Thin Python wrapper over the C ABI: torch supplies the device workspace and
the stream; every step of the tracker runs in libtpcca.so."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import TRACK_DTYPE, Geometry, Params, check


def make_geometry(geo: dict) -> Geometry:
    g = Geometry()
    g.n_sectors = int(geo["n_sectors"])
    g.n_rows = int(geo["n_rows"])
    rx = np.zeros(160, np.float32)
    rx[: g.n_rows] = np.asarray(geo["row_x"], np.float32)
    ctypes.memmove(g.row_x, rx.ctypes.data, 160 * 4)
    for k in ("bz_tesla", "tan_half_angle", "z_max", "sigma_y0", "sigma_y1", "sigma_z0",
              "sigma_z1"):
        setattr(g, k, float(geo[k]))
    return g


def default_params(**over) -> Params:
    p = Params()
    check(_lib.load().tpc_params_default(ctypes.byref(p)))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def _ptr(t) -> int:
    if isinstance(t, torch.Tensor):
        return t.data_ptr()
    return t.ctypes.data


class Tracker:
    """One tracker context on one GPU.

    geometry: dict with n_sectors, n_rows, row_x, bz_tesla, tan_half_angle,
    z_max, sigma_y0/y1/z0/z1 (see tpcgen.geometry.geometry_dict).
    """

    def __init__(self, geometry: dict, max_slots: int = 1, max_events: int = 1,
                 max_clusters: int = 4 << 20, device: str = "cuda:0", stream=None, **params):
        self.L = _lib.load()
        self.device = torch.device(device)
        self.params = default_params(max_slots=max_slots, max_events=max_events,
                                     max_clusters=int(max_clusters), **params)
        self.geometry = make_geometry(geometry)
        nbytes = self.L.tpc_workspace_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise ValueError("invalid tracker parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        # a stream of its own (graph capture needs a non-default stream)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.ctx = ctypes.c_void_p()
        rc = self.L.tpc_init_geometry(ctypes.byref(self.ctx), ctypes.byref(self.geometry),
                                      ctypes.byref(self.params), self.workspace.data_ptr(),
                                      nbytes, self.stream.cuda_stream)
        check(rc, None)
        self._keep = {}
        self._n_events = {}

    # -- staging -------------------------------------------------------------
    def load(self, slot: int, sector, row, y, z, q=None):
        """Stage one event.  Torch tensors on the GPU are used in place;
        numpy arrays are copied to the device asynchronously."""
        dev = isinstance(y, torch.Tensor) and y.is_cuda
        arrs = self._prep(sector, row, y, z, dev)
        if dev:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._hold(slot, arrs, dev)
        flags = _lib.TPC_DEVICE if dev else _lib.TPC_HOST
        n = int(arrs[2].shape[0])
        check(self.L.tpc_load_clusters(self.ctx, slot, _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]),
                                       _ptr(arrs[3]), None, n, flags), self.ctx)
        self._n_events[slot] = 1
        self._staged(slot)

    def load_batch(self, slot: int, offsets, sector, row, y, z):
        """Stage len(offsets)-1 events, concatenated, into one slot."""
        dev = isinstance(y, torch.Tensor) and y.is_cuda
        arrs = self._prep(sector, row, y, z, dev)
        offs = np.ascontiguousarray(offsets, np.int64)
        if dev:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._hold(slot, arrs + (offs,), dev)
        flags = _lib.TPC_DEVICE if dev else _lib.TPC_HOST
        check(self.L.tpc_load_batch(self.ctx, slot, len(offs) - 1, offs.ctypes.data, _ptr(arrs[0]),
                                    _ptr(arrs[1]), _ptr(arrs[2]), _ptr(arrs[3]), None, flags),
              self.ctx)
        self._n_events[slot] = len(offs) - 1
        self._staged(slot)

    def _hold(self, slot, arrs, dev):
        """Keep the staged arrays alive while the tracker's stream may read
        them.  Device tensors are marked as used on that stream (the
        allocator then does not hand their memory out before the stream's
        work is done); host arrays replaced here are released only after the
        copies queued from them have finished."""
        if dev:
            for a in arrs:
                if isinstance(a, torch.Tensor):
                    a.record_stream(self.stream)
        old = self._keep.get(slot)
        if old is not None and old[1] is not None:
            old[1].synchronize()
        self._keep[slot] = (arrs, None)

    def _staged(self, slot):
        arrs, _ = self._keep[slot]
        if not (isinstance(arrs[2], torch.Tensor) and arrs[2].is_cuda):
            ev = torch.cuda.Event()
            ev.record(self.stream)
            self._keep[slot] = (arrs, ev)

    @staticmethod
    def _prep(sector, row, y, z, dev):
        if dev:
            return (sector.to(torch.uint8).contiguous(), row.to(torch.uint8).contiguous(),
                    y.to(torch.float32).contiguous(), z.to(torch.float32).contiguous())
        return (np.ascontiguousarray(sector, np.uint8), np.ascontiguousarray(row, np.uint8),
                np.ascontiguousarray(y, np.float32), np.ascontiguousarray(z, np.float32))

    # -- tracking --------------------------------------------------------------
    def track_event(self, slot: int = 0):
        check(self.L.tpc_track_event(self.ctx, slot), self.ctx)

    def track_events(self, slots):
        """Track several staged slots, each by one replay of its HIP graph
        (captured on first use for the slot's staging)."""
        arr = np.ascontiguousarray(slots, np.int32)
        check(self.L.tpc_track_events(self.ctx, arr.ctypes.data, len(arr)), self.ctx)

    def submit(self, slot: int = 0):
        """Enqueue the tracking of a staged slot and return at once (graph
        replay if one was captured for the staging); see poll()."""
        check(self.L.tpc_submit(self.ctx, slot), self.ctx)

    def track_event_streams(self, slot: int = 0, n_streams: int = 4):
        """Per-sector launch sequences spread over n_streams streams."""
        check(self.L.tpc_track_event_streams(self.ctx, slot, n_streams), self.ctx)

    def track_sector(self, slot: int, sector: int):
        check(self.L.tpc_track_sector(self.ctx, slot, sector), self.ctx)

    def capture(self, slot: int = 0):
        """Record the slot's tracking sequence into a HIP graph."""
        check(self.L.tpc_graph_capture(self.ctx, slot), self.ctx)

    def launch(self, slot: int = 0):
        """Replay the slot's graph (asynchronous)."""
        check(self.L.tpc_graph_launch(self.ctx, slot), self.ctx)

    def poll(self, slot: int = 0) -> bool:
        """True when all work enqueued for the slot has finished."""
        rc = self.L.tpc_poll(self.ctx, slot)
        if rc == _lib.TPC_EBUSY:
            return False
        check(rc, self.ctx)
        return True

    # -- results ---------------------------------------------------------------
    def get_tracks(self, slot: int = 0, event: int = 0):
        """(tracks as a TRACK_DTYPE array, hit IDs int32) of one event."""
        nt, nh = ctypes.c_int64(0), ctypes.c_int64(0)
        rc = self.L.tpc_get_tracks(self.ctx, slot, event, None, 0, None, 0, ctypes.byref(nt),
                                   ctypes.byref(nh))
        if rc not in (_lib.TPC_OK, _lib.TPC_EOVERFLOW):
            check(rc, self.ctx)
        tracks = np.zeros(nt.value, TRACK_DTYPE)
        hits = np.zeros(nh.value, np.int32)
        check(self.L.tpc_get_tracks(self.ctx, slot, event, tracks.ctypes.data, len(tracks),
                                    hits.ctypes.data, len(hits), ctypes.byref(nt),
                                    ctypes.byref(nh)), self.ctx)
        return tracks, hits

    def get_slot_tracks(self, slot: int = 0, tracks_buf=None, hits_buf=None):
        """[(tracks, hit IDs)] of every event of the slot, as get_tracks gives
        them, read in one copy (a few synchronisations for the slot).
        tracks_buf (TRACK_DTYPE) and hits_buf (int32): optional host arrays to
        copy into, e.g. views of pinned memory, into which the copy is much
        faster; the returned arrays are then views of them, valid until they
        are written again (if they are too small, new arrays are used)."""
        ne = self._n_events.get(slot, 1)
        toff = np.zeros(ne + 1, np.uint32)
        hoff = np.zeros(ne + 1, np.uint32)
        nt, nh = ctypes.c_int64(0), ctypes.c_int64(0)
        if tracks_buf is not None and hits_buf is not None:
            assert tracks_buf.dtype == TRACK_DTYPE and hits_buf.dtype == np.int32
            rc = self.L.tpc_get_slot_tracks(self.ctx, slot, tracks_buf.ctypes.data, len(tracks_buf),
                                            hits_buf.ctypes.data, len(hits_buf), toff.ctypes.data,
                                            hoff.ctypes.data, ctypes.byref(nt), ctypes.byref(nh))
            if rc == _lib.TPC_OK:
                return [(tracks_buf[toff[e]:toff[e + 1]], hits_buf[hoff[e]:hoff[e + 1]])
                        for e in range(ne)]
            if rc != _lib.TPC_EOVERFLOW:
                check(rc, self.ctx)
        rc = self.L.tpc_get_slot_tracks(self.ctx, slot, None, 0, None, 0, toff.ctypes.data,
                                        hoff.ctypes.data, ctypes.byref(nt), ctypes.byref(nh))
        if rc not in (_lib.TPC_OK, _lib.TPC_EOVERFLOW):
            check(rc, self.ctx)
        tracks = np.zeros(nt.value, TRACK_DTYPE)
        hits = np.zeros(nh.value, np.int32)
        check(self.L.tpc_get_slot_tracks(self.ctx, slot, tracks.ctypes.data, len(tracks),
                                         hits.ctypes.data, len(hits), toff.ctypes.data,
                                         hoff.ctypes.data, ctypes.byref(nt), ctypes.byref(nh)),
              self.ctx)
        return [(tracks[toff[e]:toff[e + 1]], hits[hoff[e]:hoff[e + 1]]) for e in range(ne)]

    # -- cross-sector merger ----------------------------------------------------
    def merge(self, slot: int = 0, **over):
        """Join segments across sector boundaries (asynchronous)."""
        m = _lib.MergeParams()
        check(self.L.tpc_merge_params_default(ctypes.byref(m)))
        for k, v in over.items():
            setattr(m, k, v)
        check(self.L.tpc_merge(self.ctx, slot, ctypes.byref(m)), self.ctx)

    def get_merged(self, slot: int = 0, event: int = 0):
        """(tracks, hit IDs, segments per track) of one event after merge()."""
        nt, nh = ctypes.c_int64(0), ctypes.c_int64(0)
        rc = self.L.tpc_get_merged(self.ctx, slot, event, None, 0, None, 0, None,
                                   ctypes.byref(nt), ctypes.byref(nh))
        if rc not in (_lib.TPC_OK, _lib.TPC_EOVERFLOW):
            check(rc, self.ctx)
        tracks = np.zeros(nt.value, TRACK_DTYPE)
        hits = np.zeros(nh.value, np.int32)
        nseg = np.zeros(nt.value, np.int32)
        check(self.L.tpc_get_merged(self.ctx, slot, event, tracks.ctypes.data, len(tracks),
                                    hits.ctypes.data, len(hits), nseg.ctypes.data,
                                    ctypes.byref(nt), ctypes.byref(nh)), self.ctx)
        return tracks, hits, nseg

    def merge_links(self, slot: int, event: int, n_tracks: int):
        """Per track of get_tracks(slot, event): linked outer segment, best
        outer candidate, its chi2, output track it went into."""
        lo, bo, mi = (np.empty(n_tracks, np.int32) for _ in range(3))
        bc = np.empty(n_tracks, np.float64)
        check(self.L.tpc_get_merge_links(self.ctx, slot, event, lo.ctypes.data, bo.ctypes.data,
                                         bc.ctypes.data, mi.ctypes.data), self.ctx)
        return dict(link_out=lo, best_out=bo, best_chi2=bc, merged_into=mi)

    # -- drift-velocity calibration -------------------------------------------
    def calib_accumulate(self, slot: int, hist: torch.Tensor, z_lo: float = -20.0,
                         z_hi: float = 20.0):
        """Add the slot's tracks' beam-axis z0 to hist ([2, n_bins] int32/uint32
        on the device; asynchronous on the tracker's stream)."""
        assert hist.is_cuda and hist.dim() == 2 and hist.shape[0] == 2 and hist.is_contiguous()
        assert hist.dtype in (torch.int32,)
        # hist may have been written on torch's stream (e.g. zeroed)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        check(self.L.tpc_calib_accumulate(self.ctx, slot, hist.data_ptr(), hist.shape[1], z_lo,
                                          z_hi), self.ctx)

    def calib_correct_z(self, sector: torch.Tensor, z: torch.Tensor, eps: float):
        """Correct device cluster z in place for a drift-velocity error eps."""
        assert sector.is_cuda and z.is_cuda and sector.dtype == torch.uint8
        assert z.dtype == torch.float32 and z.is_contiguous() and sector.is_contiguous()
        # z and sector may have been written on torch's stream
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        check(self.L.tpc_calib_correct_z(self.ctx, sector.data_ptr(), z.data_ptr(), z.numel(),
                                         float(eps)), self.ctx)

    def get_links(self, slot: int, event: int, n: int):
        out = [np.empty(n, np.int32) for _ in range(4)]
        check(self.L.tpc_get_links(self.ctx, slot, event, *[o.ctypes.data for o in out]), self.ctx)
        return dict(up=out[0], dn=out[1], upc=out[2], dnc=out[3])

    def device_results(self, slot: int = 0):
        P = ctypes.c_void_p
        ptrs = [P() for _ in range(5)]
        check(self.L.tpc_device_results(self.ctx, slot, *[ctypes.byref(p) for p in ptrs]), self.ctx)
        return [p.value for p in ptrs]

    def kf_step(self, state: torch.Tensor, dx: torch.Tensor, meas: torch.Tensor):
        """One float transport + gated update per row of state[n, 20]
        (in place).  Returns (bits int32[n], chi2 float32[n])."""
        n = state.shape[0]
        cur = torch.cuda.current_stream(self.device)
        res = torch.zeros((n, 2), dtype=torch.float32, device=state.device)
        # the inputs and res were written on torch's stream; the result is
        # read there again
        self.stream.wait_stream(cur)
        for t in (state, dx, meas, res):
            t.record_stream(self.stream)
        check(self.L.tpc_kf_step_f32(self.ctx, state.data_ptr(), dx.data_ptr(), meas.data_ptr(),
                                     res.data_ptr(), n), self.ctx)
        cur.wait_stream(self.stream)
        return res[:, 0].contiguous().view(torch.int32), res[:, 1].contiguous()

    def set_profiling(self, on: bool = True):
        check(self.L.tpc_set_profiling(self.ctx, int(on)), self.ctx)

    def profile(self):
        """(stage milliseconds dict, counters dict) of the last tracked slot."""
        ms = np.zeros(len(_lib.STAGES), np.float64)
        cnt = np.zeros(len(_lib.COUNTERS), np.uint64)
        check(self.L.tpc_get_profile(self.ctx, ms.ctypes.data, cnt.ctypes.data), self.ctx)
        return (dict(zip(_lib.STAGES, ms.tolist())),
                {k: int(cnt[i]) for i, k in enumerate(_lib.COUNTERS)})

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.ctx:
            self.L.tpc_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def calib_fit(hist: torch.Tensor, out: torch.Tensor, z_max: float, eps_tracked: float = 0.0,
              z_lo: float = -20.0, z_hi: float = 20.0, stream=None):
    """Median z0 per side, the measured drift error and the estimate to adopt
    (composed with eps_tracked, the correction the events were tracked with)
    into out (4 float64 on the device), on the given stream (default: torch's
    current one); asynchronous."""
    L = _lib.load()
    assert hist.is_cuda and out.is_cuda and out.dtype == torch.float64 and out.numel() >= 4
    st = stream if stream is not None else torch.cuda.current_stream(hist.device)
    check(L.tpc_calib_fit(hist.data_ptr(), hist.shape[1], z_lo, z_hi, z_max, float(eps_tracked),
                          out.data_ptr(), st.cuda_stream))
