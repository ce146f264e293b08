"""Pins of the oracle's cross-sector merger (CPU).

The rotation between sector frames is checked against the global geometry
(trigonometry of the sector azimuths), its covariance transform against a
finite-difference Jacobian of rotate-then-transport, the 5-parameter chi2
against a dense solve, and the merges against generator truth.
"""
from __future__ import annotations

from collections import Counter

import numpy as np
import pytest

import tpcgen
import quality as Q

B = -0.00299792458 * 0.5
PACK = [(i, j) for i in range(5) for j in range(i + 1)]


def unpack(c):
    m = np.zeros((5, 5))
    for k, (i, j) in enumerate(PACK):
        m[i, j] = m[j, i] = c[k]
    return m


def pack(m):
    return np.array([m[i, j] for i, j in PACK])


def _rot_consts():
    t = float(np.float32(np.tan(np.deg2rad(10.0))))
    a = 2.0 * np.arctan(t)
    return a, np.cos(a), np.sin(a)


def _random_state(rng):
    x = rng.uniform(90.0, 240.0)
    y = rng.uniform(-0.17, 0.17) * x
    p = np.array([y, rng.uniform(-200, 200), rng.uniform(-0.6, 0.6), rng.uniform(-1, 1),
                  rng.choice([-1, 1]) / rng.uniform(0.3, 5.0)])
    a = rng.normal(size=(5, 5)) * np.array([0.05, 0.05, 1e-3, 1e-3, 1e-2])
    return x, p, pack(a @ a.T + np.diag([1e-3, 1e-3, 1e-6, 1e-6, 1e-5]))


def test_rotation_matches_global_geometry(oracle_lib):
    """(x', y', sin phi') of a state turned into the neighbouring sector's
    frame equal the global position and direction seen from that frame
    (azimuths alpha and alpha + 2 atan(tan_half_angle)), both ways."""
    rng = np.random.default_rng(11)
    ang, ca, sa = _rot_consts()
    for _ in range(300):
        x, p, C = _random_state(rng)
        alpha = np.deg2rad(rng.uniform(0, 360))
        for sgn in (1.0, -1.0):
            ok, p1, C1, x1 = oracle_lib.rotate(p, C, x, ca, sgn * sa, B)
            phi = np.arcsin(p[2])
            X = x * np.cos(alpha) - p[0] * np.sin(alpha)
            Y = x * np.sin(alpha) + p[0] * np.cos(alpha)
            a2 = alpha + sgn * ang
            xe = X * np.cos(a2) + Y * np.sin(a2)
            ye = -X * np.sin(a2) + Y * np.cos(a2)
            se = np.sin(phi - sgn * ang)
            if abs(se) > 0.95:
                assert not ok
                continue
            assert ok
            assert abs(x1 - xe) < 1e-9 and abs(p1[0] - ye) < 1e-9 and abs(p1[2] - se) < 1e-12
            assert p1[1] == p[1] and p1[3] == p[3] and p1[4] == p[4]
            ok2, p2, _, x2 = oracle_lib.rotate(p1, C1, x1, ca, -sgn * sa, B)
            assert ok2 and abs(x2 - x) < 1e-9 and abs(p2[0] - p[0]) < 1e-9
            assert abs(p2[2] - p[2]) < 1e-12


def test_rotation_covariance_is_the_transport_jacobian(oracle_lib):
    """C' = J C J^T with J the central finite-difference derivative of
    'turn the frame, then move along the track back to the unperturbed x''."""
    rng = np.random.default_rng(12)
    _, ca, sa = _rot_consts()

    def F(p, x, x_ref):
        ok, q, _, x1 = oracle_lib.rotate(p, np.zeros(15), x, ca, sa, B)
        assert ok
        ok, q, _ = oracle_lib.predict(q, np.zeros(15), x_ref - x1, B)
        assert ok
        return q

    for _ in range(50):
        x, p, C = _random_state(rng)
        ok, p0, C1, x0 = oracle_lib.rotate(p, C, x, ca, sa, B)
        if not ok:
            continue
        h = np.array([1e-4, 1e-4, 1e-7, 1e-7, 1e-6])
        J = np.zeros((5, 5))
        for i in range(5):
            e = np.zeros(5)
            e[i] = h[i]
            J[:, i] = (F(p + e, x, x0) - F(p - e, x, x0)) / (2 * h[i])
        ref = J @ unpack(C) @ J.T
        got = unpack(C1)
        scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
        assert np.max(np.abs(got - ref) / scale) < 1e-5


def test_chi2_5_is_the_dense_solve(oracle_lib):
    rng = np.random.default_rng(13)
    for _ in range(200):
        a = rng.normal(size=(5, 5))
        S = a @ a.T + 0.1 * np.eye(5)
        d = rng.normal(size=5)
        ok, c = oracle_lib.chi2_5(pack(S), d)
        assert ok
        ref = d @ np.linalg.solve(S, d)
        assert abs(c - ref) <= 1e-10 * max(1.0, ref)
    S = np.diag([1.0, 1.0, -1.0, 1.0, 1.0])
    assert not oracle_lib.chi2_5(pack(S), np.ones(5))[0]


def _majority(ev, ids):
    p, k = Counter(ev.pid[ids].tolist()).most_common(1)[0]
    return p, k / len(ids)


def _merge_case(oracle_lib, ev):
    r = oracle_lib.run_event(ev, precision=32, nthreads=8)
    m = oracle_lib.merge(r.tracks, r.hits, ev.row, ev.y, ev.z, ev.geometry())
    return r, m


@pytest.fixture(scope="module")
def peripheral(oracle_lib):
    ev = tpcgen.pbpb_event(tpcgen.seed_for(4, 100), 2000)
    return (ev,) + _merge_case(oracle_lib, ev)


def test_merges_follow_generator_truth(peripheral):
    """Linked segments belong to one particle (no wrong link allowed beyond
    0.5%); of the pairs of segments that meet the pairing conditions in
    neighbouring sectors and are their particle's only track in their
    sector (no clone or broken piece that could take the link), at least
    95% end in one output track."""
    ev, r, m = peripheral
    n = len(r.tracks)
    maj = [_majority(ev, r.track_hits(k)) for k in range(n)]
    per_sector = Counter((maj[k][0], int(r.tracks[k]["sector"])) for k in range(n))
    links = [(a, b) for a in range(n) if (b := m.link_out[a]) >= 0]
    assert len(links) > 1000
    wrong = sum(1 for a, b in links if maj[a][0] != maj[b][0] or maj[a][0] < 0)
    assert wrong <= 0.005 * len(links), wrong
    joinable, joined = 0, 0
    for a in range(n):
        for b in range(n):
            ta, tb = r.tracks[a], r.tracks[b]
            if maj[a][0] < 0 or maj[a][0] != maj[b][0]:
                continue
            if ta["sector"] // 18 != tb["sector"] // 18:
                continue
            ka, kb = ta["sector"] % 18, tb["sector"] % 18
            if not (kb == (ka + 1) % 18 or ka == (kb + 1) % 18):
                continue
            if not (0 < tb["row_in"] - ta["row_out"] <= 12):
                continue
            if (per_sector[(maj[a][0], int(ta["sector"]))] > 1
                    or per_sector[(maj[b][0], int(tb["sector"]))] > 1):
                continue
            joinable += 1
            joined += int(m.merged_into[a] == m.merged_into[b])
    assert joinable > 1000
    assert joined >= 0.95 * joinable, (joined, joinable)


def test_link_chi2_has_five_degrees_of_freedom(peripheral):
    """True links: mean chi2 near 5 (the covariances carried through the
    rotation and transport are the right size)."""
    ev, r, m = peripheral
    maj = [_majority(ev, r.track_hits(k))[0] for k in range(len(r.tracks))]
    c = [m.best_chi2[a] for a in range(len(r.tracks))
         if (b := m.link_out[a]) >= 0 and maj[a] == maj[b] and maj[a] >= 0]
    assert 4.0 < np.mean(c) < 6.5, np.mean(c)


def test_merged_track_invariants(peripheral):
    """Every input track lands in exactly one output track; a merged track's
    hits are its segments' hits, rows strictly ascending; its sector, inner
    hit and row_in are those of its innermost segment; canonical order."""
    ev, r, m = peripheral
    n = len(r.tracks)
    assert np.all(m.merged_into >= 0)
    assert len(m.tracks) == n - int((m.n_segments - 1).sum())
    members = {}
    for a in range(n):
        members.setdefault(int(m.merged_into[a]), []).append(a)
    assert np.all(np.diff(m.tracks["inner_id"]) > 0)
    for k, t in enumerate(m.tracks):
        segs = sorted(members[k], key=lambda a: r.tracks[a]["row_in"])
        assert len(segs) == m.n_segments[k]
        h = m.track_hits(k)
        assert np.array_equal(h, np.concatenate([r.track_hits(a) for a in segs]))
        assert np.all(np.diff(ev.row[h].astype(int)) > 0)
        inner = r.tracks[segs[0]]
        assert t["sector"] == inner["sector"] and t["inner_id"] == inner["inner_id"]
        assert t["row_in"] == inner["row_in"] and t["n_hits"] == len(h)
        assert t["ndf"] == 2 * t["n_hits"] - 5
        if len(segs) == 1:
            assert np.array_equal(t["par"], inner["par"]) and np.array_equal(t["cov"], inner["cov"])


def test_merged_fit_pulls_and_resolution(peripheral):
    """Merged tracks: pulls at the innermost hit against the truth of that
    cluster have unit width; the q/pT error shrinks against the innermost
    segment's own fit."""
    ev, r, m = peripheral
    sel = m.n_segments >= 2
    P = []
    shrink = []
    for k in np.nonzero(sel)[0]:
        t = m.tracks[k]
        h = m.track_hits(k)
        pid, pur = _majority(ev, h)
        h0 = int(t["inner_id"])
        if pid < 0 or pur < 0.9 or ev.pid[h0] != pid:
            continue
        d = t["par"] - ev.truth[h0]
        var = t["cov"][[0, 2, 5, 9, 14]]
        P.append(d / np.sqrt(var))
        a = int(np.nonzero(r.tracks["inner_id"] == h0)[0][0])
        shrink.append(t["cov"][14] / r.tracks[a]["cov"][14])
    P = np.array(P)
    assert len(P) > 1000
    core = np.abs(P) < 5
    rms = np.sqrt([(P[core[:, i], i] ** 2).mean() for i in range(5)])
    assert np.all((rms > 0.85) & (rms < 1.2)), rms
    assert np.all(np.abs(np.median(P, 0)) < 0.15)
    assert np.median(shrink) < 0.8


def test_nothing_to_merge_in_one_sector(oracle_lib):
    ev = tpcgen.one_sector_event()
    r, m = _merge_case(oracle_lib, ev)
    assert np.all(m.link_out < 0) and np.all(m.n_segments == 1)
    assert np.array_equal(m.tracks, r.tracks) and np.array_equal(m.hits, r.hits)


def test_membrane_crossing_segments_are_joined(oracle_lib):
    """Tracks crossing the central membrane leave a segment in sector k (A
    side) and its continuation in sector k + 18 (same azimuth, same frame):
    each such pair is linked, and the merged track holds every cluster of
    its particle (its two segments' hits), fitted across the membrane with
    parameters within 5 sigma of the truth at its innermost hit."""
    ev = tpcgen.membrane_event()
    r, m = _merge_case(oracle_lib, ev)
    n = len(r.tracks)
    maj = [_majority(ev, r.track_hits(k)) for k in range(n)]
    links = [(a, b) for a in range(n) if (b := m.link_out[a]) >= 0]
    assert len(links) == 12
    for a, b in links:
        ta, tb = r.tracks[a], r.tracks[b]
        assert maj[a][0] == maj[b][0] >= 0
        assert int(tb["sector"]) == int(ta["sector"]) + 18
        assert 0 < tb["row_in"] - ta["row_out"] <= 12
    assert len(m.tracks) == 12
    for k, t in enumerate(m.tracks):
        ids = m.hits[t["hit_off"]: t["hit_off"] + t["n_hits"]]
        p = Counter(ev.pid[ids].tolist()).most_common(1)[0][0]
        assert set(ids.tolist()) == set(np.nonzero(ev.pid == p)[0].tolist())
        tr = ev.truth[int(t["inner_id"])]
        var = np.asarray(t["cov"])[[0, 2, 5, 9, 14]]
        assert np.all(np.abs((np.asarray(t["par"]) - tr) / np.sqrt(var)) < 5.0), k


def test_boundary_jet_is_joined_by_position(oracle_lib):
    """A jet of tracks of one momentum turning across a sector boundary:
    every segment pair of the crossing passes the cuts on T and Q (tens of
    candidates per segment), so only the fitted positions and angles pick
    the partners.  Every link joins two segments of one particle, and most
    particles that left a segment on each side are joined."""
    ev = tpcgen.boundary_jet_event()
    r, m = _merge_case(oracle_lib, ev)
    n = len(r.tracks)
    maj = [_majority(ev, r.track_hits(k))[0] for k in range(n)]
    links = [(a, b) for a in range(n) if (b := m.link_out[a]) >= 0]
    assert len(links) >= 60
    assert all(maj[a] == maj[b] >= 0 for a, b in links)
    # the cuts on T and Q leave many candidates: the match decides
    sec = r.tracks["sector"].astype(int)
    crossing = Counter(maj[k] for k in range(n) if sec[k] in (0, 1) and maj[k] >= 0)
    both = [p for p, c in crossing.items()
            if {int(s) for s in sec[[k for k in range(n) if maj[k] == p]]} >= {0, 1}]
    joined = {maj[a] for a, _ in links}
    assert len(joined & set(both)) >= 0.8 * len(both), (len(joined & set(both)), len(both))
    for k in np.nonzero(m.n_segments > 1)[0]:
        ids = m.track_hits(k)
        assert Counter(ev.pid[ids].tolist()).most_common(1)[0][1] >= 0.9 * len(ids)
