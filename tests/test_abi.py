"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects bad arguments before it would touch the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1712_09416_amd import _lib
from paper_1712_09416_amd.tracker import default_params, make_geometry
import tpcgen

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "tpcca.h")


@pytest.fixture(scope="module")
def L():
    return _lib.load()


def test_exports_every_declared_symbol(L):
    src = open(HEADER).read()
    declared = set(re.findall(r"^\w[\w\s\*]*?\b(tpc_\w+)\s*\(", src, re.M))
    assert {"tpc_init_geometry", "tpc_load_clusters", "tpc_track_sector", "tpc_track_event",
            "tpc_get_tracks"} <= declared
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(_lib.EXPORTS)


def test_track_struct_layout():
    assert _lib.TRACK_DTYPE.itemsize == 216
    assert _lib.TRACK_DTYPE.fields["hit_off"][1] == 24
    assert _lib.TRACK_DTYPE.fields["par"][1] == 48


def test_params_defaults_match_oracle(L):
    from oracle.oracle import DEFAULT_PARAMS
    p = default_params()
    for k, v in DEFAULT_PARAMS.items():
        assert getattr(p, k) == pytest.approx(v), k


def test_merge_defaults_match_oracle(L):
    from oracle import oracle
    mp = _lib.MergeParams()
    assert L.tpc_merge_params_default(ctypes.byref(mp)) == _lib.TPC_OK
    om = oracle.MergeParams()
    for k, v in oracle.DEFAULT_MERGE.items():
        setattr(om, k, v)
        assert getattr(mp, k) == getattr(om, k), k      # the same float32 / int32 values
    assert ctypes.sizeof(_lib.MergeParams) == ctypes.sizeof(oracle.MergeParams) == 20


def test_workspace_bytes(L):
    p = default_params(max_clusters=1 << 20)
    a = L.tpc_workspace_bytes(ctypes.byref(p))
    p2 = default_params(max_clusters=2 << 20)
    b = L.tpc_workspace_bytes(ctypes.byref(p2))
    p3 = default_params(max_clusters=1 << 20, max_slots=3)
    c = L.tpc_workspace_bytes(ctypes.byref(p3))
    # each further slot adds the same bytes; the per-stream scratch of the
    # multi-stream path is carved once per context
    slot = (c - a) // 2
    assert 0 < a < b and c - a == 2 * slot and 0.8 * a < slot < a
    bad = default_params(max_slots=0)
    assert L.tpc_workspace_bytes(ctypes.byref(bad)) == 0
    bad = default_params(s_max=1.5)
    assert L.tpc_workspace_bytes(ctypes.byref(bad)) == 0


def _geo(**over):
    g = tpcgen.geometry.geometry_dict()
    g.update(over)
    return make_geometry(g)


def _ctx(L, ws_ptr=0x100000, **over):
    p = default_params(max_clusters=1 << 16, **over)
    need = L.tpc_workspace_bytes(ctypes.byref(p))
    ctx = ctypes.c_void_p()
    rc = L.tpc_init_geometry(ctypes.byref(ctx), ctypes.byref(_geo()), ctypes.byref(p),
                             ws_ptr, need, None)
    assert rc == _lib.TPC_OK
    return ctx, p


def test_init_rejects_bad_geometry_and_workspace(L):
    p = default_params(max_clusters=1 << 16)
    need = L.tpc_workspace_bytes(ctypes.byref(p))
    ctx = ctypes.c_void_p()
    g = _geo(n_sectors=18)
    assert L.tpc_init_geometry(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p), 0x1000, need,
                               None) == _lib.TPC_EINVAL
    assert b"36 sectors" in L.tpc_last_error(None)
    rx = tpcgen.geometry.row_x().copy()
    rx[10] = rx[9]
    g = _geo(row_x=rx)
    assert L.tpc_init_geometry(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p), 0x1000, need,
                               None) == _lib.TPC_EINVAL
    assert L.tpc_init_geometry(ctypes.byref(ctx), ctypes.byref(_geo()), ctypes.byref(p), 0x1000,
                               need - 1, None) == _lib.TPC_ENOMEM
    assert L.tpc_init_geometry(ctypes.byref(ctx), ctypes.byref(_geo()), ctypes.byref(p), None,
                               need, None) == _lib.TPC_ENOMEM
    assert L.tpc_init_geometry(None, ctypes.byref(_geo()), ctypes.byref(p), 0x1000, need,
                               None) == _lib.TPC_EINVAL


def test_calls_rejected_before_device_work(L):
    """Every check below fails on the host; no HIP call is made (there is no
    GPU here), so reaching the device would show up as TPC_EDEVICE."""
    ctx, p = _ctx(L)
    a = np.zeros(10, np.uint8)
    f = np.zeros(10, np.float32)
    P = lambda x: x.ctypes.data  # noqa: E731
    assert L.tpc_load_clusters(ctx, 1, P(a), P(a), P(f), P(f), None, 10, _lib.TPC_HOST) == _lib.TPC_EINVAL
    assert L.tpc_load_clusters(ctx, -1, P(a), P(a), P(f), P(f), None, 10, _lib.TPC_HOST) == _lib.TPC_EINVAL
    assert L.tpc_load_clusters(ctx, 0, P(a), P(a), P(f), P(f), None, -1, _lib.TPC_HOST) == _lib.TPC_EINVAL
    assert L.tpc_load_clusters(ctx, 0, P(a), P(a), P(f), P(f), None, (1 << 16) + 1,
                               _lib.TPC_HOST) == _lib.TPC_ENOMEM
    assert L.tpc_load_clusters(ctx, 0, None, P(a), P(f), P(f), None, 10, _lib.TPC_HOST) == _lib.TPC_EINVAL
    assert L.tpc_load_clusters(ctx, 0, P(a), P(a), P(f), P(f), None, 10, 7) == _lib.TPC_EINVAL
    offs = np.array([0, 5, 3], np.int64)
    assert L.tpc_load_batch(ctx, 0, 2, offs.ctypes.data, P(a), P(a), P(f), P(f), None,
                            _lib.TPC_HOST) == _lib.TPC_EINVAL          # decreasing / too many events
    offs = np.array([1, 5], np.int64)
    assert L.tpc_load_batch(ctx, 0, 1, offs.ctypes.data, P(a), P(a), P(f), P(f), None,
                            _lib.TPC_HOST) == _lib.TPC_EINVAL
    assert L.tpc_track_event(ctx, 0) == _lib.TPC_ESTATE
    assert L.tpc_track_event(ctx, 3) == _lib.TPC_EINVAL
    assert L.tpc_track_sector(ctx, 0, 0) == _lib.TPC_ESTATE
    assert L.tpc_track_event_streams(ctx, 0, 4) == _lib.TPC_ESTATE
    assert L.tpc_track_event_streams(ctx, 0, 0) == _lib.TPC_EINVAL
    assert L.tpc_track_event_streams(ctx, 0, 9) == _lib.TPC_EINVAL
    assert L.tpc_track_event_streams(ctx, 2, 4) == _lib.TPC_EINVAL
    mp = _lib.MergeParams()
    assert L.tpc_merge_params_default(ctypes.byref(mp)) == _lib.TPC_OK
    assert L.tpc_merge(ctx, 0, ctypes.byref(mp)) == _lib.TPC_ESTATE
    assert L.tpc_merge(ctx, 0, None) == _lib.TPC_EINVAL
    for k, v in (("passes", 0), ("s_max", 1.0), ("row_gap", 0), ("chi2_max", 0.0),
                 ("step_max", 0.05)):
        bad = _lib.MergeParams()
        L.tpc_merge_params_default(ctypes.byref(bad))
        setattr(bad, k, v)
        assert L.tpc_merge(ctx, 0, ctypes.byref(bad)) == _lib.TPC_EINVAL, k
    assert L.tpc_get_merged(ctx, 0, 0, None, 0, None, 0, None, ctypes.byref(ctypes.c_int64()),
                            ctypes.byref(ctypes.c_int64())) == _lib.TPC_ESTATE
    assert L.tpc_get_merge_links(ctx, 0, 0, None, None, None, None) == _lib.TPC_ESTATE
    nt, nh = ctypes.c_int64(), ctypes.c_int64()
    assert L.tpc_get_tracks(ctx, 0, 0, None, 0, None, 0, ctypes.byref(nt),
                            ctypes.byref(nh)) == _lib.TPC_ESTATE
    assert L.tpc_get_tracks(ctx, 0, 0, None, 5, None, 0, ctypes.byref(nt),
                            ctypes.byref(nh)) == _lib.TPC_EINVAL
    assert L.tpc_get_tracks(ctx, 0, 0, None, -1, None, 0, None, None) == _lib.TPC_EINVAL
    # the whole slot's output: offset arrays required, buffer sizes, state
    off = np.zeros(2, np.uint32)
    assert L.tpc_get_slot_tracks(None, 0, None, 0, None, 0, off.ctypes.data, off.ctypes.data,
                                 None, None) == _lib.TPC_EINVAL
    assert L.tpc_get_slot_tracks(ctx, 0, None, 0, None, 0, None, off.ctypes.data,
                                 None, None) == _lib.TPC_EINVAL
    assert L.tpc_get_slot_tracks(ctx, 0, None, -1, None, 0, off.ctypes.data, off.ctypes.data,
                                 None, None) == _lib.TPC_EINVAL
    assert L.tpc_get_slot_tracks(ctx, 0, None, 4, None, 0, off.ctypes.data, off.ctypes.data,
                                 None, None) == _lib.TPC_EINVAL
    assert L.tpc_get_slot_tracks(ctx, 7, None, 0, None, 0, off.ctypes.data, off.ctypes.data,
                                 None, None) == _lib.TPC_EINVAL
    assert L.tpc_get_slot_tracks(ctx, 0, None, 0, None, 0, off.ctypes.data, off.ctypes.data,
                                 None, None) == _lib.TPC_ESTATE
    assert L.tpc_get_links(ctx, 0, 0, None, None, None, None) == _lib.TPC_ESTATE
    assert L.tpc_kf_step_f32(ctx, None, None, None, None, 5) == _lib.TPC_EINVAL
    assert L.tpc_kf_step_f32(ctx, None, None, None, None, 0) == _lib.TPC_OK
    assert L.tpc_last_error(ctx)
    assert L.tpc_track_event(None, 0) == _lib.TPC_EINVAL
    # batched graph replay and the serving entry: list and state checks
    one = np.array([0], np.int32)
    assert L.tpc_track_events(ctx, None, 1) == _lib.TPC_EINVAL
    assert L.tpc_track_events(ctx, one.ctypes.data, 0) == _lib.TPC_EINVAL
    assert L.tpc_track_events(ctx, one.ctypes.data, 1) == _lib.TPC_EINVAL       # default stream
    assert L.tpc_submit(ctx, 0) == _lib.TPC_ESTATE
    assert L.tpc_submit(ctx, 5) == _lib.TPC_EINVAL
    assert L.tpc_submit(None, 0) == _lib.TPC_EINVAL
    # drift fit: histogram, range and the eps the events were tracked with
    h = np.zeros(8, np.uint32)
    o = np.zeros(4, np.float64)
    assert L.tpc_calib_fit(None, 4, -1.0, 1.0, 250.0, 0.0, o.ctypes.data, None) == _lib.TPC_EINVAL
    assert L.tpc_calib_fit(h.ctypes.data, 4, 1.0, -1.0, 250.0, 0.0, o.ctypes.data, None) == _lib.TPC_EINVAL
    assert L.tpc_calib_fit(h.ctypes.data, 4, -1.0, 1.0, 250.0, 0.7, o.ctypes.data, None) == _lib.TPC_EINVAL
    assert L.tpc_calib_fit(h.ctypes.data, 4, -1.0, 1.0, 250.0, float("nan"), o.ctypes.data,
                           None) == _lib.TPC_EINVAL


def test_track_events_checks_every_slot_first(L):
    """A bad entry anywhere in the list is refused before any slot is
    tracked (a non-null stream handle makes the list checks reachable; no
    call below reaches the device)."""
    p = default_params(max_clusters=1 << 10, max_slots=3)
    need = L.tpc_workspace_bytes(ctypes.byref(p))
    ctx = ctypes.c_void_p()
    assert L.tpc_init_geometry(ctypes.byref(ctx), ctypes.byref(_geo()), ctypes.byref(p), 0x100000,
                               need, 0x1000) == _lib.TPC_OK
    for bad, rc in (([0, 3], _lib.TPC_EINVAL), ([1, 1], _lib.TPC_EINVAL), ([2, -1], _lib.TPC_EINVAL),
                    ([0, 1], _lib.TPC_ESTATE), ([0, 1, 2, 0], _lib.TPC_EINVAL)):
        arr = np.array(bad, np.int32)
        assert L.tpc_track_events(ctx, arr.ctypes.data, len(arr)) == rc, bad


def test_track_regions_sized_for_n_min_track(L):
    """Every output track owns at least n_min_track hits that no other
    track owns, so a slot of N clusters needs room for N / n_min_track
    tracks: the workspace grows as n_min_track falls, and values below 3
    are refused."""
    sizes = []
    for nmt in (10, 5, 3):
        p = default_params(max_clusters=1 << 20, n_min_track=nmt)
        sizes.append(L.tpc_workspace_bytes(ctypes.byref(p)))
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    # the track regions (par, cov, owned hits and rows, merger buffers) are
    # the only part that changes: about 1.8 kB per track of capacity
    per_track = (sizes[2] - sizes[0]) / ((1 << 20) // 3 - (1 << 20) // 10)
    assert 1500 < per_track < 2500, per_track
    bad = default_params(n_min_track=2)
    assert L.tpc_workspace_bytes(ctypes.byref(bad)) == 0


def test_tracklet_regions_sized_for_n_min_chain(L):
    """A start hit heads its own cleaned chain of >= n_min_chain hits and
    the chains are disjoint, so a slot of N clusters needs room for
    N / n_min_chain tracklets: the workspace shrinks as n_min_chain grows;
    values outside 3..159 are refused."""
    sizes = [L.tpc_workspace_bytes(ctypes.byref(default_params(max_clusters=1 << 20, n_min_chain=c)))
             for c in (3, 4, 8)]
    assert sizes[0] > sizes[1] > sizes[2] > 0
    for bad in (2, 160):
        assert L.tpc_workspace_bytes(ctypes.byref(default_params(n_min_chain=bad))) == 0, bad


def test_noalloc_checks_before_device_work(L):
    """The allocation-free entry refuses, before any device call, a missing
    status array, an event too large for its fixed workspace and bad
    params (an event of 400,000 clusters needs ~145 MB of workspace)."""
    g = make_geometry(tpcgen.geometry.geometry_dict())
    p = default_params()
    a = np.zeros(16, np.uint32)
    ptr = a.ctypes.data
    big = 400_000
    args = (ptr, ptr, ptr, ptr, big, ptr, 4, ptr, 4)
    assert L.tpc_track_event_noalloc(ctypes.byref(g), ctypes.byref(p), *args, None, None) == \
        _lib.TPC_EINVAL
    assert L.tpc_track_event_noalloc(ctypes.byref(g), ctypes.byref(p), *args, ptr, None) == \
        _lib.TPC_ENOMEM
    assert b"allocation-free" in L.tpc_last_error(None)
    bad = default_params(n_min_chain=2)
    small = (ptr, ptr, ptr, ptr, 10, ptr, 4, ptr, 4)
    assert L.tpc_track_event_noalloc(ctypes.byref(g), ctypes.byref(bad), *small, ptr, None) == \
        _lib.TPC_EINVAL
    assert L.tpc_track_event_noalloc(ctypes.byref(g), ctypes.byref(p), ptr, ptr, ptr, ptr, -1,
                                     ptr, 4, ptr, 4, ptr, None) == _lib.TPC_EINVAL


def test_batch_event_limit(L):
    ctx, p = _ctx(L, max_events=4)
    a = np.zeros(10, np.uint8)
    f = np.zeros(10, np.float32)
    offs = np.zeros(6, np.int64)
    assert L.tpc_load_batch(ctx, 0, 5, offs.ctypes.data, a.ctypes.data, a.ctypes.data,
                            f.ctypes.data, f.ctypes.data, None, _lib.TPC_HOST) == _lib.TPC_EINVAL


def test_every_package_module_imports():
    """Every module of the package and the generator imports on the CPU
    (the binding loads the library lazily; nothing here touches a GPU)."""
    import importlib
    import pkgutil
    import paper_1712_09416_amd as pkg
    import tpcgen as gen
    for mod in (pkg, gen):
        for info in pkgutil.iter_modules(mod.__path__):
            if info.name.startswith("lib"):          # the built shared library itself
                continue
            importlib.import_module(f"{mod.__name__}.{info.name}")


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits
    non-zero before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
