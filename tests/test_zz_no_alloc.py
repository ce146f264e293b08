"""The allocation-free entry point, tpc_track_event_noalloc, called through
the C ABI: its tracks and hit IDs are identical to those of the path with a
caller workspace (tpc_load_clusters + tpc_track_event + tpc_get_tracks) on
the same events, on calls in a row with smaller inputs each time (the
library's array keeps the previous call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

import tpcgen
from paper_1712_09416_amd import _lib
from paper_1712_09416_amd.tracker import Tracker, default_params, make_geometry

pytestmark = pytest.mark.gpu

REC = _lib.TRACK_DTYPE.itemsize


def say(*a):
    print(*a, flush=True)


def _inputs(ev, dev):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]


def _with_workspace(ev, dev):
    trk = Tracker(ev.geometry(), max_clusters=max(ev.n, 16))
    trk.load(0, *_inputs(ev, dev))
    trk.track_event(0)
    tracks, hits = trk.get_tracks(0)
    trk.close()
    return tracks, hits


def _noalloc(ev, dev, stream, max_tracks, max_hits):
    L = _lib.load()
    ins = _inputs(ev, dev)
    out_t = torch.zeros(max(1, max_tracks) * REC, dtype=torch.uint8, device=dev)
    out_h = torch.full((max(1, max_hits),), -7, dtype=torch.int32, device=dev)
    status = torch.full((4,), -1, dtype=torch.int32, device=dev)
    g = make_geometry(ev.geometry())
    p = default_params()
    stream.wait_stream(torch.cuda.current_stream(dev))
    rc = L.tpc_track_event_noalloc(ctypes.byref(g), ctypes.byref(p), ins[0].data_ptr(),
                                   ins[1].data_ptr(), ins[2].data_ptr(), ins[3].data_ptr(), ev.n,
                                   out_t.data_ptr(), max_tracks, out_h.data_ptr(), max_hits,
                                   status.data_ptr(), stream.cuda_stream)
    assert rc == _lib.TPC_OK, L.tpc_last_error(None)
    stream.synchronize()
    st = status.cpu().numpy().view(np.uint32)
    nt, nh = int(st[0]), int(st[1])
    kt, kh = min(nt, max_tracks), min(nh, max_hits)
    tracks = out_t.cpu().numpy()[: kt * REC].view(_lib.TRACK_DTYPE)
    hits = out_h.cpu().numpy()[:kh]
    return tracks, hits, st


def _same(a, b):
    assert len(a) == len(b), (len(a), len(b))
    for k in _lib.TRACK_DTYPE.names:
        assert np.array_equal(a[k], b[k]), k


def test_noalloc_equals_workspace_path():
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    events = [tpcgen.one_sector_event(), tpcgen.pp_event(), tpcgen.tiny_event(7, n_tracks=4)]
    sizes = [ev.n for ev in events]
    assert sizes[0] > sizes[1] > sizes[2] > 0
    for ev in events:
        say(f"no-alloc: {ev.name} event, {ev.n} clusters")
        ref_t, ref_h = _with_workspace(ev, dev)
        tracks, hits, st = _noalloc(ev, dev, stream, len(ref_t) + 5, len(ref_h) + 5)
        assert st[0] == len(ref_t) and st[1] == len(ref_h) and st[2] == 0 and st[3] == 0, st
        _same(tracks, ref_t)
        assert np.array_equal(hits, ref_h)
        say(f"no-alloc: {len(tracks)} tracks identical")


def test_noalloc_output_bounds_and_empty_event():
    """Output arrays smaller than the event's tracks: the first max_tracks
    records and max_hits IDs are written, the status carries the full counts
    and flag bit 3; an empty event gives no tracks."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    ev = tpcgen.pp_event()
    ref_t, ref_h = _with_workspace(ev, dev)
    assert len(ref_t) > 4
    tracks, hits, st = _noalloc(ev, dev, stream, 3, 20)
    assert st[0] == len(ref_t) and st[1] == len(ref_h) and st[2] == 8, st
    _same(tracks, ref_t[:3])
    assert np.array_equal(hits, ref_h[:20])
    empty = tpcgen.pp_event()
    for k in ("sector", "row", "y", "z"):
        setattr(empty, k, getattr(empty, k)[:0])
    tracks, hits, st = _noalloc(empty, dev, stream, 4, 4)
    assert len(tracks) == 0 and len(hits) == 0 and st[0] == 0 and st[1] == 0 and st[2] == 0, st
