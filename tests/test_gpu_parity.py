"""GPU parity: the HIP tracker (through the C ABI) against the CPU oracle.

Bar: links and track hit lists identical to the oracle's float run (the
same decisions in the same precision and operation order); track
parameters / covariances identical to the oracle's (both refit in double
from identical float seeds) and within 1e-4 relative (floors 10 cm, 10 cm,
0.1, 0.1, 0.1) / 1e-3 of sqrt(C_ii C_jj) of the double replay.
"""
import ctypes

import numpy as np
import pytest

import tpcgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FLOOR = np.array([10.0, 10.0, 0.1, 0.1, 0.1])
ORACLE_THREADS = 16          # host threads for the oracle runs
PACK = [(i, j) for i in range(5) for j in range(i + 1)]


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def gpu_run(ev, dev, mode="event", tracker=None, links=True, geometry=None, **params):
    from paper_1712_09416_amd import Tracker
    trk = tracker or Tracker(geometry or ev.geometry(), max_clusters=max(ev.n, 4096), **params)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    trk.load(0, *ins)
    if mode == "event":
        trk.track_event(0)
    elif mode == "sectors":
        for s in range(36):
            trk.track_sector(0, s)
    else:                                   # "streams<n>"
        trk.track_event_streams(0, int(mode[7:]))
    tracks, hits = trk.get_tracks(0)
    lk = trk.get_links(0, 0, ev.n) if links else None
    if tracker is None:
        trk.close()
    return tracks, hits, lk


def compare_links(lk, ref, sel=None):
    for k in ("up", "dn", "upc", "dnc"):
        g = lk[k]
        o = getattr(ref, k)
        if sel is not None:
            g = g[sel]
            o = np.where(o >= 0, sel[np.maximum(o, 0)], -1)
        bad = np.count_nonzero(g != o)
        assert bad == 0, f"{k}: {bad} of {len(g)} links differ"


def compare_tracks(tracks, hits, ref, sel=None):
    assert len(tracks) == len(ref.tracks), (len(tracks), len(ref.tracks))
    rh = ref.hits if sel is None else sel[ref.hits]
    assert np.array_equal(hits, rh)
    for k in ("n_hits", "row_in", "row_out", "ndf", "hit_off", "x_ref"):
        assert np.array_equal(tracks[k], ref.tracks[k]), k
    inner = ref.tracks["inner_id"] if sel is None else sel[ref.tracks["inner_id"]]
    start = ref.tracks["start_id"] if sel is None else sel[ref.tracks["start_id"]]
    assert np.array_equal(tracks["inner_id"], inner)
    assert np.array_equal(tracks["start_id"], start)
    for k in ("par", "cov", "chi2"):
        d = np.count_nonzero(tracks[k] != ref.tracks[k])
        assert d == 0, f"{k}: {d} values differ from the oracle's (expected bitwise)"


def compare_replay(tracks, rep, min_hits=0):
    """The replay bar on the tracks of at least min_hits hits."""
    keep = tracks["n_hits"] >= min_hits
    tracks, rep = tracks[keep], rep[keep]
    pe = np.abs(tracks["par"] - rep["par"]) / np.maximum(np.abs(rep["par"]), FLOOR)
    assert pe.max() <= 1e-4, pe.max()
    diag = rep["cov"][:, [0, 2, 5, 9, 14]]
    den = np.stack([np.sqrt(diag[:, i] * diag[:, j]) for i, j in PACK], 1)
    ce = np.abs(tracks["cov"] - rep["cov"]) / den
    assert ce.max() <= 1e-3, ce.max()


# ---------------------------------------------------------------------------

def test_kf_step_bitwise(dev, oracle_lib):
    """One float transport + gated update on 10^6 random states: identical
    bits on the GPU and in the oracle's float primitives (state, accept
    flags and chi2)."""
    from paper_1712_09416_amd import Tracker
    rng = np.random.default_rng(42)
    n = 1_000_000
    st = np.zeros((n, 20), np.float32)
    st[:, 0] = rng.uniform(-40, 40, n)
    st[:, 1] = rng.uniform(-250, 250, n)
    st[:, 2] = rng.uniform(-0.9, 0.9, n)
    st[:, 3] = rng.uniform(-1.2, 1.2, n)
    st[:, 4] = rng.uniform(-10, 10, n)
    A = rng.normal(size=(n, 5, 5)) * np.array([0.3, 0.4, 0.03, 0.03, 0.5])
    C = A @ A.transpose(0, 2, 1) + np.diag([1e-3, 1e-3, 1e-5, 1e-5, 1e-3])
    st[:, 5:] = np.stack([C[:, i, j] for i, j in PACK], 1).astype(np.float32)
    del A, C
    dx = rng.choice(np.array([-1.5, -1.0, -0.75, 0.75, 1.0, 1.5], np.float32), n)
    meas = np.zeros((n, 4), np.float32)
    meas[:, 0] = st[:, 0] + dx * st[:, 2] + rng.normal(size=n).astype(np.float32) * 0.5
    meas[:, 1] = st[:, 1] + dx * st[:, 3] + rng.normal(size=n).astype(np.float32) * 0.5
    meas[:, 2] = rng.uniform(0.005, 0.05, n)
    meas[:, 3] = rng.uniform(0.005, 0.05, n)
    trk = Tracker(tpcgen.geometry.geometry_dict(), max_clusters=1024)
    gs = torch.from_numpy(st.copy()).to(dev)
    bits, chi2 = trk.kf_step(gs, torch.from_numpy(dx).to(dev), torch.from_numpy(meas).to(dev))
    gs, bits, chi2 = gs.cpu().numpy(), bits.cpu().numpy(), chi2.cpu().numpy()
    trk.close()
    b = np.float32(-0.00299792458 * np.float64(np.float32(0.5)))
    ost, obits, ochi = oracle_lib.kf_steps_f32(st, dx, meas, b, 0.95, 16.0)
    assert (obits & 1).mean() > 0.5 and (obits & 2).mean() > 0.2
    assert np.array_equal(bits, obits), np.count_nonzero(bits != obits)
    same = (gs.view(np.uint32) == ost.view(np.uint32)).all(axis=1)
    same &= chi2.view(np.uint32) == ochi.view(np.uint32)
    assert same.all(), f"{np.count_nonzero(~same)} of {n} steps differ"


def test_one_sector_event(dev, oracle_lib):
    ev = tpcgen.one_sector_event()
    say(f"one-sector event: {ev.n} clusters")
    tracks, hits, lk = gpu_run(ev, dev)
    ref = oracle_lib.run_event(ev, precision=32, replay=True)
    compare_links(lk, ref)
    compare_tracks(tracks, hits, ref)
    compare_replay(tracks, ref.replay)


def test_pp_event_plain_and_fused(dev, oracle_lib):
    ev = tpcgen.pp_event()
    say(f"pp event: {ev.n} clusters")
    ref = oracle_lib.run_event(ev, precision=32, replay=True)
    for mode in ("event", "sectors"):
        tracks, hits, lk = gpu_run(ev, dev, mode=mode)
        compare_links(lk, ref)
        compare_tracks(tracks, hits, ref)
        compare_replay(tracks, ref.replay)


@pytest.mark.parametrize("seed_off", [0, 1, 2])
def test_pbpb_small_events(dev, oracle_lib, seed_off):
    ev = tpcgen.pbpb_event(tpcgen.seed_for(2) + 50 + seed_off, 500 + 700 * seed_off)
    say(f"pbpb event {seed_off}: {ev.n} clusters")
    tracks, hits, lk = gpu_run(ev, dev)
    ref = oracle_lib.run_event(ev, precision=32, replay=True, nthreads=8)
    compare_links(lk, ref)
    compare_tracks(tracks, hits, ref)
    compare_replay(tracks, ref.replay)


def test_central_event_all_sectors(dev, oracle_lib):
    """The central Pb-Pb-shaped event at full size on the GPU (all sectors in
    one launch per step, the bench's configuration) against the oracle on the
    whole event: links, hit lists, parameters and covariances identical, and
    within the bar of the double replay."""
    ev = tpcgen.central_event()
    say(f"central event: {ev.n} clusters")
    tracks, hits, lk = gpu_run(ev, dev)
    ref = oracle_lib.run_event(ev, precision=32, replay=True, nthreads=ORACLE_THREADS)
    compare_links(lk, ref)
    compare_tracks(tracks, hits, ref)
    compare_replay(tracks, ref.replay)
    assert np.all(np.diff(tracks["inner_id"]) > 0)
    assert len(np.unique(hits)) == len(hits)
    say(f"central event: {len(tracks)} tracks, {len(hits)} hits, identical to the oracle")
    # the plain per-sector launch sequence (each launch sized by its sector)
    tracks, hits, lk = gpu_run(ev, dev, mode="sectors")
    compare_links(lk, ref)
    compare_tracks(tracks, hits, ref)
    say("central event, per-sector launches: identical to the oracle")


def test_batch_equals_single_events(dev, oracle_lib):
    """Events tracked together in one slot (one cluster-error model for the
    whole slot: the Pb-Pb one) give exactly the oracle's tracks of each
    event, and so their single-event results; the whole slot read in one
    copy gives each event the same block."""
    from paper_1712_09416_amd import Tracker
    evs = [tpcgen.pbpb_event(tpcgen.seed_for(3, e), m) for e, m in enumerate([50, 900, 3000])]
    evs.insert(1, tpcgen.pp_event())
    empty = tpcgen.pp_event()
    for k in ("sector", "row", "y", "z"):
        setattr(empty, k, getattr(empty, k)[:0])
    evs.insert(2, empty)
    offs = np.concatenate([[0], np.cumsum([e.n for e in evs])])
    cat = [np.concatenate([getattr(e, k) for e in evs]) for k in ("sector", "row", "y", "z")]
    geo = evs[0].geometry()
    trk = Tracker(geo, max_events=8, max_clusters=int(offs[-1]) + 16)
    trk.load_batch(0, offs, *[torch.from_numpy(a).to(dev) for a in cat])
    trk.track_event(0)
    whole = trk.get_slot_tracks(0)              # every event in one copy
    assert len(whole) == len(evs)
    # into caller buffers (pinned host memory), large enough or not
    from paper_1712_09416_amd._lib import TRACK_DTYPE
    for n_t, n_h in ((1 << 14, 1 << 20), (3, 5)):
        tb_buf = torch.empty(n_t * TRACK_DTYPE.itemsize, dtype=torch.uint8,
                             pin_memory=True).numpy().view(TRACK_DTYPE)
        hb_buf = torch.empty(n_h, dtype=torch.int32, pin_memory=True).numpy()
        again = trk.get_slot_tracks(0, tb_buf, hb_buf)
        for (t1, h1), (t2, h2) in zip(again, whole):
            assert np.array_equal(t1, t2) and np.array_equal(h1, h2)
    for e, ev in enumerate(evs):
        tb, hb = trk.get_tracks(0, e)
        assert np.all(tb["event"] == e)
        assert np.array_equal(whole[e][0], tb) and np.array_equal(whole[e][1], hb), e
        ref = oracle_lib.run(ev.sector, ev.row, ev.y, ev.z, geo, precision=32, nthreads=ORACLE_THREADS)
        compare_tracks(tb, hb, ref)
        ts, hs, _ = gpu_run(ev, dev, links=False, geometry=geo)
        assert np.array_equal(hb, hs)
        for k in ("n_hits", "inner_id", "hit_off", "par", "cov", "chi2", "sector"):
            assert np.array_equal(tb[k], ts[k]), (e, k)
    # buffers too small: the counts and offsets still come back
    toff = np.zeros(len(evs) + 1, np.uint32)
    hoff = np.zeros(len(evs) + 1, np.uint32)
    nt, nh = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = trk.L.tpc_get_slot_tracks(trk.ctx, 0, None, 0, None, 0, toff.ctypes.data,
                                   hoff.ctypes.data, ctypes.byref(nt), ctypes.byref(nh))
    assert rc == -3                             # TPC_EOVERFLOW
    assert nt.value == sum(len(w[0]) for w in whole) == toff[-1]
    assert nh.value == sum(len(w[1]) for w in whole) == hoff[-1]
    trk.close()


def test_events_in_flight_match_oracle(dev, oracle_lib):
    """Events in flight as in the bench's timed region: three trackers, each
    with its own stream and workspace, take six events round-robin with no
    synchronisation between the launches; every event's tracks equal the
    oracle's."""
    from paper_1712_09416_amd import Tracker
    evs = [tpcgen.pbpb_event(tpcgen.seed_for(2) + 200 + e, m)
           for e, m in enumerate([1500, 300, 2500, 800, 60, 1200])]
    geo = evs[0].geometry()
    cap = max(e.n for e in evs)
    trks = [Tracker(geo, max_slots=2, max_clusters=cap) for _ in range(3)]
    ins = [[torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (e.sector, e.row, e.y, e.z)]
           for e in evs]
    for i, e in enumerate(evs):                  # slot i // 3 of tracker i % 3
        t = trks[i % 3]
        t.load(i // 3, *ins[i])
        t.track_event(i // 3)
    for i, e in enumerate(evs):
        tracks, hits = trks[i % 3].get_tracks(i // 3)
        ref = oracle_lib.run(e.sector, e.row, e.y, e.z, geo, precision=32, nthreads=ORACLE_THREADS)
        compare_tracks(tracks, hits, ref)
    for t in trks:
        t.close()


def test_full_batch_graph_matches_oracle(dev, oracle_lib):
    """The bench's batch at full size (64 Pb-Pb-shaped events of
    multiplicity 50-15000, 31.5M clusters, 2304 sectors in one launch per
    step), tracked by tpc_track_events (captured on the first call,
    replayed from its HIP graph on the second): every event's tracks, hit
    lists, parameters and covariances identical to the oracle's run of that
    event alone."""
    from paper_1712_09416_amd import Tracker
    from tpcgen import parallel
    mult = tpcgen.batch_multiplicities(64)
    gen = parallel.generate([("batch", (e, int(m))) for e, m in enumerate(mult)])
    offs = np.concatenate([[0], np.cumsum([len(d["y"]) for d in gen])]).astype(np.int64)
    say(f"batch: {len(gen)} events, {offs[-1]} clusters")
    cat = [torch.from_numpy(np.concatenate([d[k] for d in gen])).to(dev)
           for k in ("sector", "row", "y", "z")]
    geo = tpcgen.geometry.geometry_dict(gen[0]["sigma"])
    trk = Tracker(geo, max_events=len(gen), max_clusters=int(offs[-1]))
    trk.load_batch(0, offs, *cat)
    trk.track_events([0])
    trk.track_events([0])
    ntk = 0
    for e, d in enumerate(gen):
        tb, hb = trk.get_tracks(0, e)
        ref = oracle_lib.run(d["sector"], d["row"], d["y"], d["z"], geo, precision=32,
                             nthreads=ORACLE_THREADS)
        try:
            compare_tracks(tb, hb, ref)
        except AssertionError as err:
            raise AssertionError(f"event {e} ({len(d['y'])} clusters): {err}") from None
        ntk += len(tb)
    say(f"batch: {ntk} tracks, every event identical to the oracle")
    trk.close()


def test_edge_cases(dev):
    from paper_1712_09416_amd import Tracker, TpcError
    geo = tpcgen.geometry.geometry_dict()
    trk = Tracker(geo, max_clusters=1 << 14)

    def run(sector, row, y, z):
        trk.load(0, *[torch.from_numpy(np.asarray(a)).to(dev) for a in
                      (np.asarray(sector, np.uint8), np.asarray(row, np.uint8),
                       np.asarray(y, np.float32), np.asarray(z, np.float32))])
        trk.track_event(0)
        return trk.get_tracks(0)

    t, h = run([], [], [], [])
    assert len(t) == 0 and len(h) == 0
    t, h = run([3], [10], [1.0], [5.0])
    assert len(t) == 0
    # a row full of clusters and nothing else
    rng = np.random.default_rng(1)
    t, h = run(np.zeros(3000), np.full(3000, 70), rng.uniform(-20, 20, 3000), rng.uniform(0, 250, 3000))
    assert len(t) == 0
    # one straight noise-free track plus uniform noise, on the C side
    x = tpcgen.geometry.row_x()
    sec = np.full(159, 20)
    t, h = run(sec, np.arange(159), 0.05 * x, -0.5 * x)
    assert len(t) == 1 and t[0]["n_hits"] == 159 and t[0]["sector"] == 20
    # invalid clusters are reported
    with pytest.raises(TpcError) as e:
        run([0, 1], [10, 200], [0.0, 0.0], [1.0, 1.0])
    assert "invalid" in str(e.value)
    with pytest.raises(TpcError):
        run([0, 40], [10, 10], [0.0, 0.0], [1.0, 1.0])
    with pytest.raises(TpcError):
        run([0, 1], [10, 10], [np.nan, 0.0], [1.0, 1.0])
    # more than 4096 clusters in one pad row: refused, the rest stays sane
    t = None
    with pytest.raises(TpcError) as e:
        run(np.zeros(5000), np.full(5000, 30), rng.uniform(-10, 10, 5000), rng.uniform(0, 250, 5000))
    assert "4096" in str(e.value)
    # the context is still usable afterwards
    t, h = run(sec, np.arange(159), 0.05 * x, -0.5 * x)
    assert len(t) == 1
    # capacity of one cluster: every pad row empty or nearly so, each with
    # its largest number of bins (the bin table's worst case per cluster)
    small = Tracker(geo, max_clusters=1)
    for args in (([], [], [], []), ([7], [80], [2.0], [30.0])):
        small.load(0, *[torch.from_numpy(np.asarray(a, d)).to(dev) for a, d in
                        zip(args, (np.uint8, np.uint8, np.float32, np.float32))])
        small.track_event(0)
        t, h = small.get_tracks(0)
        assert len(t) == 0 and len(h) == 0
    small.close()
    trk.close()


def edge_rows_event(seed=20261203):
    """Straight tracks placed at the row range's ends, plus seeded uniform
    noise in their sectors: one ending at the last pad row, one starting at
    pad row 0, one of exactly ten hits, one of runs of six hits with an
    empty row between (steps without a hit in every fit), and a nine-hit one
    on the C side that is too short to become a track."""
    from tpcgen.events import Event
    rng = np.random.default_rng(seed)
    x = tpcgen.geometry.row_x()
    S, R, Y, Z = [], [], [], []

    def line(sec, rows, a, b):
        rows = np.asarray(rows)
        S.append(np.full(len(rows), sec))
        R.append(rows)
        Y.append(a * x[rows])
        Z.append(b * x[rows])

    line(4, np.arange(145, 159), 0.02, 0.3)
    line(5, np.arange(0, 15), -0.03, 0.2)
    line(6, np.arange(60, 70), 0.01, 0.5)
    line(7, [r for r in range(20, 110) if (r - 20) % 7 != 6], 0.04, 0.4)
    line(24, np.arange(150, 159), -0.01, -0.6)
    for sec in (4, 5, 6, 7, 24):
        rr = rng.integers(0, 159, 300)
        S.append(np.full(300, sec))
        R.append(rr)
        Y.append(rng.uniform(-0.15, 0.15, 300) * x[rr])
        Z.append(rng.uniform(0, 250, 300) * (-1.0 if sec >= 18 else 1.0))
    p = rng.permutation(sum(len(a) for a in S))
    s, r, y, z = (np.concatenate(a)[p] for a in (S, R, Y, Z))
    n = len(s)
    return Event("edge_rows", seed, s.astype(np.uint8), r.astype(np.uint8), y.astype(np.float32),
                 z.astype(np.float32), np.ones(n, np.float32), np.full(n, -1, np.int32),
                 np.full(n, -1, np.int32), np.full((n, 5), np.nan), (0.1, 0.0, 0.15, 0.0))


def test_tracks_at_row_range_ends(dev, oracle_lib):
    """Tracklets that run to the last pad row or down to row 0, a track of
    the minimum length and fits with empty rows between hits: links, hit
    lists and parameters identical to the oracle's, in the fused and the
    per-sector launch sequences."""
    ev = edge_rows_event()
    say(f"edge-rows event: {ev.n} clusters")
    ref = oracle_lib.run_event(ev, precision=32, replay=True)
    rows = sorted(zip(ref.tracks["n_hits"].tolist(), ref.tracks["row_in"].tolist(),
                      ref.tracks["row_out"].tolist()))
    assert rows == [(10, 60, 69), (14, 145, 158), (15, 0, 14), (78, 20, 109)], rows
    from paper_1712_09416_amd import Tracker
    for mode in ("event", "sectors"):
        trk = Tracker(ev.geometry(), max_clusters=4096)
        tracks, hits, lk = gpu_run(ev, dev, mode=mode, tracker=trk)
        compare_links(lk, ref)
        compare_tracks(tracks, hits, ref)
        compare_replay(tracks, ref.replay)
        # the merger's outward walk over these tracks (empty rows included)
        trk.merge(0)
        merge_case(trk, 0, 0, ev, oracle_lib)
        trk.close()


def test_repeat_runs_identical(dev):
    ev = tpcgen.pbpb_event(tpcgen.seed_for(2) + 77, 2000)
    a = gpu_run(ev, dev, links=False)
    b = gpu_run(ev, dev, links=False)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])


def test_graph_replays_match_eager(dev):
    """The captured tracking graph, replayed several times with other eager
    work in between, gives the eager result every time (and so does the
    merger run on a replayed slot); a slot re-staged with another shape is
    refused."""
    from paper_1712_09416_amd import Tracker, TpcError
    ev = tpcgen.pbpb_event(tpcgen.seed_for(2) + 90, 1500)
    trk = Tracker(ev.geometry(), max_clusters=ev.n + 100)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    trk.load(0, *ins)
    trk.track_event(0)
    ref_t, ref_h = trk.get_tracks(0)
    trk.merge(0)
    ref_m = trk.get_merged(0)
    trk.load(0, *ins)
    trk.capture(0)
    for k in range(4):
        junk = torch.randn(1 << 20, device=dev).sum().item()       # eager work between replays
        assert np.isfinite(junk)
        trk.launch(0)
        t, h = trk.get_tracks(0)
        assert np.array_equal(h, ref_h), k
        assert np.array_equal(t, ref_t), k
        if k % 2 == 1:                  # the merger runs on a replayed slot too
            trk.merge(0)
            for a, b in zip(trk.get_merged(0), ref_m):
                assert np.array_equal(a, b), k
        trk.load(0, *ins)
    other = [a[:-10].contiguous() for a in ins]
    trk.load(0, *other)
    with pytest.raises(TpcError):
        trk.launch(0)
    trk.close()


def test_serving_results_equal_alone(dev, oracle_lib):
    """Requests served with continuous batching over several streams (and
    with the plain one-at-a-time path) give each event exactly the oracle's
    tracks of that event alone; every third request arrives in pinned host
    tensors (transferred from there) and the others in numpy arrays (staged),
    so batches mix the two."""
    from paper_1712_09416_amd.serve import Server, Request, poisson_arrivals
    pool = [tpcgen.pbpb_event(tpcgen.seed_for(4, e), m) for e, m in enumerate([60, 300, 900, 150])]
    geo = pool[0].geometry()
    refs = [oracle_lib.run(ev.sector, ev.row, ev.y, ev.z, geo, precision=32, nthreads=ORACLE_THREADS)
            for ev in pool]
    pinned = [[torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
               for a in (ev.sector, ev.row, ev.y, ev.z)] for ev in pool]
    arr = poisson_arrivals(40, 2000.0, seed=5)
    reqs = [Request(float(arr[i]), *(pinned[i % 4] if i % 3 == 0 else
                                     (pool[i % 4].sector, pool[i % 4].row, pool[i % 4].y,
                                      pool[i % 4].z)), tag=str(i % 4)) for i in range(40)]
    for plain in (False, True):
        srv = Server(geo, n_streams=3, max_events=4, cap_clusters=600_000, plain=plain)
        st = srv.run(reqs, collect=True)
        srv.close()
        say(f"serving plain={plain}: {st.summary()}")
        assert st.n_requests == 40
        for i, (t, h) in enumerate(st.results):
            try:
                compare_tracks(t, h, refs[i % 4])
            except AssertionError as err:
                raise AssertionError(f"plain={plain} request {i}: {err}") from None


def test_autotune_knobs_keep_tracks(dev, oracle_lib):
    """Every launch shape the autotuner tries (grid bin sizes, extreme ones
    included; tracklet block size; window hits and hit-list rows read per
    round trip) gives the same tracks (the tuner raises otherwise), and the
    tuned shape's tracks are the oracle's."""
    from paper_1712_09416_amd import Tracker
    from paper_1712_09416_amd.autotune import autotune
    evs = [tpcgen.pbpb_event(tpcgen.seed_for(3, 900 + e), m) for e, m in enumerate([120, 700, 40])]
    geo = evs[0].geometry()
    offs = np.concatenate([[0], np.cumsum([e.n for e in evs])]).astype(np.int64)
    cat = [torch.from_numpy(np.concatenate([getattr(e, k) for e in evs])).to(dev)
           for k in ("sector", "row", "y", "z")]
    knobs = {"bin_target": (2.0, 0.5, 8.0, 64.0), "bin_min_edge": (2.0, 0.5, 10.0)}
    res = autotune(geo, offs, *cat, knobs=knobs, reps=1)
    say(f"autotune: best {res['best']}, {len(res['ms'])} shapes")
    assert len(res["ms"]) == 12 + 2 + 2 + 2
    trk = Tracker(geo, max_events=len(evs), max_clusters=int(offs[-1]), **res["best"])
    trk.load_batch(0, offs, *cat)
    trk.track_event(0)
    for e, ev in enumerate(evs):
        tb, hb = trk.get_tracks(0, e)
        compare_tracks(tb, hb, oracle_lib.run(ev.sector, ev.row, ev.y, ev.z, geo, precision=32,
                                              nthreads=ORACLE_THREADS))
    trk.close()


def test_multi_stream_sectors_equal_fused(dev, oracle_lib):
    """Per-sector launch sequences spread over several streams (sectors in
    flight together) give exactly the oracle's tracks and links, for a
    single event, and the fused path's tracks for a batch slot."""
    from paper_1712_09416_amd import Tracker
    ev = tpcgen.pbpb_event(tpcgen.seed_for(2) + 91, 1200)
    geo = ev.geometry()
    ref = oracle_lib.run_event(ev, precision=32, nthreads=ORACLE_THREADS)
    assert len(ref.tracks) > 100
    trk = Tracker(geo, max_clusters=ev.n)
    for ns in (1, 3, 8):
        t, h, lk = gpu_run(ev, dev, mode=f"streams{ns}", tracker=trk)
        compare_links(lk, ref)
        compare_tracks(t, h, ref)
    trk.close()
    evs = [tpcgen.pbpb_event(tpcgen.seed_for(3, 950 + e), m) for e, m in enumerate([300, 60, 900])]
    offs = np.concatenate([[0], np.cumsum([e.n for e in evs])]).astype(np.int64)
    cat = [torch.from_numpy(np.concatenate([getattr(e, k) for e in evs])).to(dev)
           for k in ("sector", "row", "y", "z")]
    trk = Tracker(geo, max_events=3, max_clusters=int(offs[-1]))
    trk.load_batch(0, offs, *cat)
    trk.track_event_streams(0, 4)
    for e, ev in enumerate(evs):
        t, h = trk.get_tracks(0, e)
        compare_tracks(t, h, oracle_lib.run_event(ev, precision=32, nthreads=ORACLE_THREADS))
    trk.close()


def short_segments_event(seed=20261204):
    """Straight noise-free 5-hit segments from the origin in one sector,
    spaced 8 cm apart in y and z at every row they share, in 15 bands of
    rows: ~2,600 tracks of 5 hits, one per 5 clusters, twice the number of
    tracks a region sized for >= 10 hits per track holds."""
    from tpcgen.events import Event
    x = tpcgen.geometry.row_x()
    S, R, Y, Z = [], [], [], []
    for band in range(15):
        rows = np.arange(10 * band + 2, 10 * band + 7)
        xm = x[rows].mean()
        ymax = xm * np.tan(np.deg2rad(10.0)) - 2.0
        for yc in np.arange(-ymax, ymax, 8.0):
            for zc in np.arange(4.0, 245.0, 8.0):
                a, b = yc / xm, zc / xm
                if np.any(np.abs(b * x[rows]) > 248.0):
                    continue
                S.append(np.full(5, 3))
                R.append(rows)
                Y.append(a * x[rows])
                Z.append(b * x[rows])
    rng = np.random.default_rng(seed)
    p = rng.permutation(sum(len(a) for a in S))
    s, r, y, z = (np.concatenate(a)[p] for a in (S, R, Y, Z))
    n = len(s)
    return Event("short_segments", seed, s.astype(np.uint8), r.astype(np.uint8), y.astype(np.float32),
                 z.astype(np.float32), np.ones(n, np.float32), np.full(n, -1, np.int32),
                 np.full(n, -1, np.int32), np.full((n, 5), np.nan), (0.1, 0.0, 0.15, 0.0))


def test_min_track_length_three_matches_oracle(dev, oracle_lib):
    """n_min_track = n_min_tracklet = n_min_chain = 3 (the smallest
    accepted): every tracklet and track region is sized for n / 3 entries,
    so the fused, per-sector and
    multi-stream sequences stay inside their sectors' regions; links, hit
    lists and parameters identical to the oracle run with the same cuts, and
    the merger over these short segments identical to the oracle's.
    The replay bar is checked on the tracks of ten hits or more: below
    that, the oracle's own three-pass double refit from the float seed
    differs from the all-double replay by up to 1.1e-3 (3-4 hit tracks,
    5 parameters from 6-8 measurements, where the linearisation point still
    moves between passes), which is the method's, not the GPU's."""
    from paper_1712_09416_amd import Tracker
    ev = tpcgen.pbpb_event(tpcgen.seed_for(2) + 93, 800)
    cuts = dict(n_min_track=3, n_min_tracklet=3, n_min_chain=3)
    ref = oracle_lib.run_event(ev, precision=32, replay=True, nthreads=ORACLE_THREADS,
                               params=oracle_lib.make_params(**cuts))
    short = int((ref.tracks["n_hits"] < 10).sum())
    say(f"n_min_track=3: {len(ref.tracks)} tracks, {short} with fewer than 10 hits")
    assert short > 0
    trk = Tracker(ev.geometry(), max_clusters=ev.n, **cuts)
    for mode in ("event", "sectors", "streams4"):
        tracks, hits, lk = gpu_run(ev, dev, mode=mode, tracker=trk)
        compare_links(lk, ref)
        compare_tracks(tracks, hits, ref)
        compare_replay(tracks, ref.replay, min_hits=10)
    # the merger over segments as short as three hits
    trk.merge(0)
    mref = merge_case(trk, 0, 0, ev, oracle_lib)
    assert (mref.n_segments > 1).sum() > 0
    trk.close()
    # one sector holding a track per five clusters
    ev = short_segments_event()
    ref = oracle_lib.run_event(ev, precision=32, params=oracle_lib.make_params(**cuts))
    say(f"short segments: {ev.n} clusters, {len(ref.tracks)} tracks")
    assert len(ref.tracks) > ev.n // 10 + 1
    trk = Tracker(ev.geometry(), max_clusters=ev.n, **cuts)
    for mode in ("event", "sectors", "streams2"):
        tracks, hits, lk = gpu_run(ev, dev, mode=mode, tracker=trk)
        compare_links(lk, ref)
        compare_tracks(tracks, hits, ref)
    trk.close()


# cuts and detector constants other than the defaults: (params, geometry)
NONDEFAULT = {
    "tight": (dict(nf_window=2.0, nf_mmax=9.0, chi2_max=9.0, k_win=3.0, w_max=3.0, n_gap=3), {}),
    "loose": (dict(nf_window=4.5, nf_mmax=25.0, chi2_max=25.0, k_win=5.0, w_max=8.0, s_max=0.9,
                   c_s0=0.5, c_t0=2.0, c_q0=50.0, m_edge=0.5, m_z=2.0, n_gap=8,
                   n_min_tracklet=8, n_min_track=8, n_min_chain=5), {}),
    "reversed_field": ({}, dict(bz_tesla=np.float32(-0.5))),
    "sigma_and_drift": ({}, dict(sigma_y0=np.float32(0.15), sigma_y1=np.float32(0.05),
                                 sigma_z0=np.float32(0.2), sigma_z1=np.float32(0.05),
                                 z_max=np.float32(245.0))),
}


@pytest.mark.parametrize("case", sorted(NONDEFAULT))
def test_nondefault_constants_match_oracle(dev, oracle_lib, case):
    """Every cut and detector constant reaches the kernels from the
    parameters and the geometry (none is compiled in): with tighter and
    looser cuts than the defaults, the magnetic field reversed, and another
    cluster-error model and drift length, links, hit lists and parameters
    equal the oracle's run with the same values."""
    cuts, g = NONDEFAULT[case]
    ev = tpcgen.pbpb_event(tpcgen.seed_for(2) + 77, 800)
    geo = dict(ev.geometry(), **g)
    ref = oracle_lib.run(ev.sector, ev.row, ev.y, ev.z, geo, precision=32, replay=True,
                         nthreads=ORACLE_THREADS, params=oracle_lib.make_params(**cuts))
    say(f"{case}: {ev.n} clusters, {len(ref.tracks)} tracks")
    assert len(ref.tracks) > 1000 and ref.replay_bad == 0
    tracks, hits, lk = gpu_run(ev, dev, geometry=geo, **cuts)
    compare_links(lk, ref)
    compare_tracks(tracks, hits, ref)
    compare_replay(tracks, ref.replay)


def test_track_events_and_submit(dev, oracle_lib):
    """tpc_track_events over three slots (captured on the first call, then
    replayed; a re-staged slot is captured again) and tpc_submit (graph
    replay when the slot has one for its staging, else the eager sequence):
    every slot's tracks identical to the oracle's."""
    from paper_1712_09416_amd import Tracker
    evs = [tpcgen.pbpb_event(tpcgen.seed_for(3, 970 + e), m) for e, m in enumerate([200, 700, 60, 400])]
    geo = evs[0].geometry()
    refs = [oracle_lib.run_event(ev, precision=32, nthreads=ORACLE_THREADS) for ev in evs]
    trk = Tracker(geo, max_slots=3, max_clusters=max(ev.n for ev in evs))
    ins = [[torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
           for ev in evs]

    def check(slot, k):
        t, h = trk.get_tracks(slot)
        try:
            compare_tracks(t, h, refs[k])
        except AssertionError as err:
            raise AssertionError(f"slot {slot} (event {k}): {err}") from None

    for slot in range(3):
        trk.load(slot, *ins[slot])
    for _ in range(2):
        trk.track_events([2, 0, 1])
        for slot in range(3):
            check(slot, slot)
    trk.load(1, *ins[3])                       # another shape: captured again
    trk.track_events([1])
    check(1, 3)
    trk.load(1, *ins[3])                       # same staging: submit replays the graph
    trk.submit(1)
    while not trk.poll(1):
        pass
    check(1, 3)
    fresh = Tracker(geo, max_clusters=evs[1].n)
    fresh.load(0, *ins[1])                     # no graph: submit runs the eager sequence
    fresh.submit(0)
    t, h = fresh.get_tracks(0)
    compare_tracks(t, h, refs[1])
    fresh.close()
    trk.close()


# ---------------------------------------------------------------------------
# cross-sector merger

def compare_merged(gt, gh, gseg, ref):
    assert len(gt) == len(ref.tracks), (len(gt), len(ref.tracks))
    assert np.array_equal(gh, ref.hits)
    assert np.array_equal(gseg, ref.n_segments)
    for k in ("sector", "n_hits", "row_in", "row_out", "ndf", "hit_off", "inner_id", "start_id",
              "x_ref"):
        assert np.array_equal(gt[k], ref.tracks[k]), k
    for k in ("par", "cov", "chi2"):
        d = np.count_nonzero(gt[k] != ref.tracks[k])
        assert d == 0, f"merged {k}: {d} values differ from the oracle's (expected bitwise)"


def as_oracle_tracks(tracks, oracle_lib):
    """The library's track records in the oracle's record layout (by field
    name; numpy would assign structured records by position)."""
    out = np.zeros(len(tracks), oracle_lib.TRACK_DTYPE)
    for k in out.dtype.names:
        if k in tracks.dtype.names:
            out[k] = tracks[k]
    return out


def merge_case(trk, slot, event, ev, oracle_lib, geometry=None):
    tracks, hits = trk.get_tracks(slot, event)
    gt, gh, gseg = trk.get_merged(slot, event)
    lk = trk.merge_links(slot, event, len(tracks))
    ref = oracle_lib.merge(as_oracle_tracks(tracks, oracle_lib), hits, ev.row, ev.y, ev.z,
                           geometry or ev.geometry())
    say(f"merge {ev.name}: {len(tracks)} -> {len(gt)} tracks, {int((gseg > 1).sum())} chains")
    assert np.array_equal(lk["best_out"], ref.best_out)
    assert np.array_equal(lk["best_chi2"][ref.best_out >= 0], ref.best_chi2[ref.best_out >= 0])
    assert np.array_equal(lk["link_out"], ref.link_out)
    assert np.array_equal(lk["merged_into"], ref.merged_into)
    compare_merged(gt, gh, gseg, ref)
    return ref


@pytest.mark.parametrize("kind", ["pp", "peripheral", "central", "membrane", "jet"])
def test_merge_matches_oracle(dev, oracle_lib, kind):
    """Merged tracks, hit lists, segment counts, links and best-candidate
    chi2 bit-identical to the oracle's merger run on the same tracks (which
    are themselves bit-identical to the oracle's tracker); the membrane
    workload's twelve segment pairs across z = 0 are all joined.  In the
    boundary jet every segment pair of the crossing passes the T and Q cuts,
    so a wave's four tracks queue well over 64 pairs (the LDS queue is
    evaluated full many times, as well as at the end)."""
    from paper_1712_09416_amd import Tracker
    ev = {"pp": lambda: tpcgen.pp_event(),
          "peripheral": lambda: tpcgen.pbpb_event(tpcgen.seed_for(4, 101), 2000),
          "central": lambda: tpcgen.central_event(),
          "membrane": lambda: tpcgen.membrane_event(),
          "jet": lambda: tpcgen.boundary_jet_event()}[kind]()
    trk = Tracker(ev.geometry(), max_clusters=ev.n)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    trk.load(0, *ins)
    trk.track_event(0)
    trk.merge(0)
    ref = merge_case(trk, 0, 0, ev, oracle_lib)
    if kind in ("peripheral", "central"):
        assert (ref.n_segments > 1).sum() > 100
    if kind == "membrane":
        assert len(ref.tracks) == 12 and np.all(ref.n_segments == 2)
    if kind == "jet":
        assert (ref.n_segments > 1).sum() >= 60
    # a second merge of the same tracking gives the same output
    trk.merge(0)
    gt, gh, gseg = trk.get_merged(0, 0)
    compare_merged(gt, gh, gseg, ref)
    trk.close()


@pytest.mark.parametrize("over", [dict(chi2_max=10.0, row_gap=6, step_max=1.0, passes=2, s_max=0.99),
                                  dict(chi2_max=60.0, row_gap=20, step_max=4.0, passes=4)],
                         ids=["tight", "loose"])
def test_merge_params_match_oracle(dev, oracle_lib, over):
    """Merge cuts other than the defaults (match chi2, row gap, transport
    step, refit passes, |sin phi| bound) reach the kernels: the merged
    output equals the oracle's merger with the same values."""
    from paper_1712_09416_amd import Tracker
    ev = tpcgen.pbpb_event(tpcgen.seed_for(4, 101), 2000)
    trk = Tracker(ev.geometry(), max_clusters=ev.n)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    trk.load(0, *ins)
    trk.track_event(0)
    trk.merge(0, **over)
    tracks, hits = trk.get_tracks(0, 0)
    gt, gh, gseg = trk.get_merged(0, 0)
    lk = trk.merge_links(0, 0, len(tracks))
    ref = oracle_lib.merge(as_oracle_tracks(tracks, oracle_lib), hits, ev.row, ev.y, ev.z,
                           ev.geometry(), **over)
    say(f"merge {over}: {len(tracks)} -> {len(gt)} tracks")
    assert (ref.n_segments > 1).sum() > 50
    assert np.array_equal(lk["best_out"], ref.best_out)
    assert np.array_equal(lk["best_chi2"][ref.best_out >= 0], ref.best_chi2[ref.best_out >= 0])
    assert np.array_equal(lk["link_out"], ref.link_out)
    assert np.array_equal(lk["merged_into"], ref.merged_into)
    compare_merged(gt, gh, gseg, ref)
    trk.close()


def test_merge_pair_list_overflow_matches_oracle(dev, oracle_lib):
    """The first pair pass lists the compatible pairs for the second, two per
    track of the slot's capacity; beyond that the second pass walks the
    candidates again.  With the match cut opened (chi2 <= 1e6) on the
    boundary jet and a capacity sized for 30-hit tracks, the candidate pairs
    (3,700) outnumber the list (~1,700): the merged output still equals the
    oracle's merger with the same cut."""
    from paper_1712_09416_amd import Tracker
    ev = tpcgen.boundary_jet_event()
    trk = Tracker(ev.geometry(), max_clusters=ev.n, n_min_track=30)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    trk.load(0, *ins)
    trk.track_event(0)
    trk.merge(0, chi2_max=1e6)
    tracks, hits = trk.get_tracks(0, 0)
    sec = tracks["sector"].astype(int)
    ri, ro = tracks["row_in"].astype(int), tracks["row_out"].astype(int)
    n_cand = 0
    for a in range(len(tracks)):
        side, k = divmod(sec[a], 18)
        nb = {side * 18 + (k + 1) % 18, side * 18 + (k + 17) % 18, (1 - side) * 18 + k}
        n_cand += int(np.count_nonzero(np.isin(sec, list(nb)) & (ri > ro[a]) & (ri <= ro[a] + 12)))
    cap = 2 * (ev.n // 30 + 36)
    say(f"pair list: {n_cand} candidate pairs, room for {cap}")
    assert n_cand > 1.5 * cap
    gt, gh, gseg = trk.get_merged(0, 0)
    lk = trk.merge_links(0, 0, len(tracks))
    ref = oracle_lib.merge(as_oracle_tracks(tracks, oracle_lib), hits, ev.row, ev.y, ev.z,
                           ev.geometry(), chi2_max=1e6)
    assert (ref.n_segments > 1).sum() > 30
    assert np.array_equal(lk["best_out"], ref.best_out)
    assert np.array_equal(lk["best_chi2"][ref.best_out >= 0], ref.best_chi2[ref.best_out >= 0])
    assert np.array_equal(lk["link_out"], ref.link_out)
    compare_merged(gt, gh, gseg, ref)
    trk.close()


def test_merge_batch_equals_single(dev, oracle_lib):
    """Merging a batch slot gives each event its own single-event merge."""
    from paper_1712_09416_amd import Tracker
    evs = [tpcgen.pbpb_event(tpcgen.seed_for(3, 960 + e), m) for e, m in enumerate([400, 50, 1500])]
    geo = evs[0].geometry()
    offs = np.concatenate([[0], np.cumsum([e.n for e in evs])]).astype(np.int64)
    cat = [torch.from_numpy(np.concatenate([getattr(e, k) for e in evs])).to(dev)
           for k in ("sector", "row", "y", "z")]
    trk = Tracker(geo, max_events=3, max_clusters=int(offs[-1]))
    trk.load_batch(0, offs, *cat)
    trk.track_event(0)
    trk.merge(0)
    for e, ev in enumerate(evs):
        merge_case(trk, 0, e, ev, oracle_lib, geometry=geo)
    trk.close()


def test_merge_edge_cases(dev, oracle_lib):
    """No tracks; one sector only (nothing to merge); merge refused before
    tracking and after re-staging."""
    from paper_1712_09416_amd import Tracker, TpcError
    geo = tpcgen.geometry.geometry_dict()
    trk = Tracker(geo, max_clusters=50_000)
    z = torch.zeros(0, device=dev)
    u8 = torch.zeros(0, dtype=torch.uint8, device=dev)
    trk.load(0, u8, u8, z, z)
    with pytest.raises(TpcError):
        trk.merge(0)
    trk.track_event(0)
    trk.merge(0)
    gt, gh, gseg = trk.get_merged(0, 0)
    assert len(gt) == 0 and len(gh) == 0
    ev = tpcgen.one_sector_event()
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    trk.load(0, *ins)
    with pytest.raises(TpcError):
        trk.get_merged(0, 0)
    trk.track_event(0)
    trk.merge(0)
    tracks, hits = trk.get_tracks(0)
    gt, gh, gseg = trk.get_merged(0, 0)
    assert len(gt) == len(tracks) and np.array_equal(gh, hits) and np.all(gseg == 1)
    for k in tracks.dtype.names:
        assert np.array_equal(gt[k], tracks[k]), k
    merge_case(trk, 0, 0, ev, oracle_lib)
    trk.close()


# ---------------------------------------------------------------------------
# drift-velocity calibration

def test_calibration_matches_oracle(dev, oracle_lib):
    """Histogram of beam-axis z0 (integers), fitted medians and eps, and the
    z correction: bit-identical to the oracle's on the same tracks."""
    from paper_1712_09416_amd import Tracker
    from paper_1712_09416_amd.tracker import calib_fit
    ev = tpcgen.distort_drift(tpcgen.pbpb_event(tpcgen.seed_for(4, 103), 2000), 0.003)
    geo = ev.geometry()
    trk = Tracker(geo, max_clusters=ev.n)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ev.sector, ev.row, ev.y, ev.z)]
    trk.load(0, *ins)
    trk.track_event(0)
    hist = torch.zeros((2, 4000), dtype=torch.int32, device=dev)
    trk.calib_accumulate(0, hist)
    tracks, _ = trk.get_tracks(0)
    ref = oracle_lib.calib_histogram(as_oracle_tracks(tracks, oracle_lib), geo)
    trk.synchronize()
    h = hist.cpu().numpy().view(np.uint32)
    assert np.array_equal(h, ref)
    out = torch.zeros(4, dtype=torch.float64, device=dev)
    calib_fit(hist, out, 250.0, 0.0, stream=trk.stream)
    trk.synchronize()
    got = out.cpu().numpy()
    exp = np.array(oracle_lib.calib_fit(ref, 250.0))
    say(f"calibration: {got} (oracle {exp})")
    assert np.array_equal(got, exp)
    assert abs(got[2] - 0.003) < 1e-4 and got[3] == got[2]
    # the same histogram read as events tracked after a correction of 0.001
    calib_fit(hist, out, 250.0, 0.001, stream=trk.stream)
    trk.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got, np.array(oracle_lib.calib_fit(ref, 250.0, eps_tracked=0.001)))
    z = ins[3].clone()
    trk.calib_correct_z(ins[0], z, float(got[2]))
    trk.synchronize()
    assert np.array_equal(z.cpu().numpy(), oracle_lib.drift_correct(ev.sector, ev.z, float(got[2]), 250.0))
    # an empty side gives NaN
    h1 = torch.zeros((2, 4000), dtype=torch.int32, device=dev)
    h1[0, 2000] = 3
    calib_fit(h1, out, 250.0, 0.0, stream=trk.stream)
    trk.synchronize()
    got = out.cpu().numpy()
    exp = oracle_lib.calib_fit(h1.cpu().numpy().view(np.uint32), 250.0)
    assert got[0] == exp[0] and np.isnan(got[1]) and np.isnan(got[2]) and np.isnan(got[3])
    trk.close()


def test_calibration_side_task_converges_while_serving(dev):
    """Events served with a 0.4% drift-velocity error: the side task's fits
    (polled, never waited for) bring the correction to the true value, and
    every event is still served."""
    from paper_1712_09416_amd.calib import DriftCalibration
    from paper_1712_09416_amd.serve import Server, Request, poisson_arrivals
    pool = [tpcgen.distort_drift(tpcgen.pbpb_event(tpcgen.seed_for(4, 110 + e), 1500), 0.004)
            for e in range(6)]
    geo = pool[0].geometry()
    arr = poisson_arrivals(90, 400.0, seed=9)
    reqs = [Request(float(arr[i]), pool[i % 6].sector, pool[i % 6].row, pool[i % 6].y,
                    pool[i % 6].z) for i in range(90)]
    cal = DriftCalibration(250.0, every=12, device=dev)
    srv = Server(geo, n_streams=3, max_events=4, cap_clusters=2_000_000, calib=cal)
    st = srv.run(reqs)
    srv.close()
    say(f"calibration fits: {cal.history}; serving {st.summary()}")
    assert st.n_requests == 90
    assert len(cal.history) >= 2
    assert abs(cal.eps - 0.004) < 2e-4, cal.eps



def test_multiple_scattering_matches_oracle(dev, oracle_lib):
    """With the scattering noise on (X0 = 3000 cm, scattered tracks): links,
    hit lists and parameters bit-identical to the oracle; within the bar of
    the double replay."""
    from tpcgen import events as E
    ev = E.ms_sector_event(1005, 200, x0_cm=3000.0)
    ref = oracle_lib.run_event(ev, precision=32, replay=True,
                               params=oracle_lib.make_params(x0_cm=3000.0))
    assert ref.replay_bad == 0 and len(ref.tracks) > 100
    tracks, hits, lk = gpu_run(ev, dev, x0_cm=3000.0)
    compare_links(lk, ref)
    compare_tracks(tracks, hits, ref)
    compare_replay(tracks, ref.replay)
