"""The synthetic-event generator: geometry, reproducibility, truth records.

The generator is the ground truth behind the oracle's pins, so its helix
crossings are checked here against the circle and z-line equations directly.
"""
import numpy as np
import pytest

import tpcgen
from tpcgen import geometry as G


def test_row_radii():
    x = G.row_x()
    assert x.dtype == np.float32 and x.shape == (159,)
    assert np.isclose(x[0], 85.225) and np.isclose(x[62], 85.225 + 0.75 * 62)
    assert np.isclose(x[63], 135.1) and np.isclose(x[126], 198.1)
    assert np.isclose(x[127], 199.35) and np.isclose(x[158], 245.85)
    d = np.diff(x.astype(np.float64))
    assert np.all(d > 0)
    assert set(np.round(d, 3)) <= {0.75, 1.0, 1.5, 49.875 - 48.125, 135.1 - 131.725, 199.35 - 198.1}


def test_seed_reproducible():
    a = tpcgen.one_sector_event()
    b = tpcgen.one_sector_event()
    for k in ("sector", "row", "y", "z", "pid"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    c = tpcgen.one_sector_event(tpcgen.seed_for(0) + 1)
    assert c.n != a.n or not np.array_equal(a.y, c.y)


def _circle_check(ev):
    """Every signal cluster's true local position lies on its particle's
    helix: on the circle in the transverse plane and on the z line."""
    p = ev.particles
    sig = ev.pid >= 0
    pid = ev.pid[sig]
    sec = ev.sector[sig].astype(np.int64)
    x = G.row_x()[ev.row[sig]].astype(np.float64)
    ytrue = ev.truth[sig, 0]
    ztrue = ev.truth[sig, 1]
    a = G.sector_alpha(sec)
    X = x * np.cos(a) - ytrue * np.sin(a)
    Y = x * np.sin(a) + ytrue * np.cos(a)
    R = p["pt"][pid] / (G.C_LIGHT * G.BZ_TESLA)
    h = -np.sign(p["charge"][pid])
    xc = p["vx"][pid] - h * R * np.sin(p["phi"][pid])
    yc = p["vy"][pid] + h * R * np.cos(p["phi"][pid])
    assert np.allclose(np.hypot(X - xc, Y - yc), R, rtol=0, atol=1e-8 * R.max())
    # z along the helix: z - vz = T * (arc length), arc length = R * turning angle
    ang = np.arctan2(Y - yc, X - xc)
    ang0 = np.arctan2(p["vy"][pid] - yc, p["vx"][pid] - xc)
    turn = np.mod(h * (ang - ang0), 2 * np.pi)          # turning angle from the vertex
    T = np.sinh(p["eta"][pid])
    l = (ztrue - p["vz"][pid]) / np.where(T == 0, np.nan, T)
    # arc length is the turning angle times R, modulo whole turns
    frac = np.mod(l / R - turn + 1e-9, 2 * np.pi) - 1e-9
    assert np.nanmax(np.abs(frac)) < 1e-6
    # acceptance and side
    assert np.all(np.abs(ytrue) <= x * np.tan(np.deg2rad(10.0)) + 1e-9)
    assert np.all((ztrue >= 0) == (sec < 18))
    assert np.all(np.abs(ztrue) <= G.Z_MAX)


def test_helix_crossings_one_sector():
    _circle_check(tpcgen.one_sector_event())


def test_helix_crossings_pbpb_secondaries_loopers():
    _circle_check(tpcgen.pbpb_event(tpcgen.seed_for(2) + 7, 300))


def test_truth_sin_phi_is_local_direction():
    """s = sin(phi - alpha) follows from the circle: s = (x - xc_loc) / (h R)
    with xc_loc the circle centre's local x."""
    ev = tpcgen.one_sector_event()
    p = ev.particles
    sig = np.nonzero(ev.pid >= 0)[0]
    pid = ev.pid[sig]
    a = G.sector_alpha(ev.sector[sig].astype(np.int64))
    R = p["pt"][pid] / (G.C_LIGHT * G.BZ_TESLA)
    h = -np.sign(p["charge"][pid])
    xc = -h * R * np.sin(p["phi"][pid])
    yc = h * R * np.cos(p["phi"][pid])
    xloc_c = xc * np.cos(a) + yc * np.sin(a)
    x = G.row_x()[ev.row[sig]].astype(np.float64)
    assert np.allclose((x - xloc_c) / (h * R), ev.truth[sig, 2], atol=1e-12)


def test_truth_of_returning_legs():
    """A returning looper leg, followed towards larger x, has its direction
    turned by pi: sin phi, tan lambda and q/pT all change sign, and
    consecutive crossings of the leg step x upwards with y consistent with
    that direction (dy/dx = tan phi)."""
    ev = tpcgen.pbpb_event(tpcgen.seed_for(2) + 11, 400)
    sig = np.nonzero((ev.pid >= 0) & (ev.leg % 2 == 1))[0]
    assert len(sig) > 100
    key = ev.pid[sig].astype(np.int64) * 1000 + ev.sector[sig].astype(np.int64) * 200 + ev.row[sig]
    key = key * 4 + ev.leg[sig]
    o = np.argsort(key)
    s, k = sig[o], key[o]
    nxt = np.nonzero(np.diff(k) == 4)[0]      # same leg, next row
    a, b = s[nxt], s[nxt + 1]
    x = G.row_x().astype(np.float64)
    dydx = (ev.truth[b, 0] - ev.truth[a, 0]) / (x[ev.row[b]] - x[ev.row[a]])
    sm = 0.5 * (ev.truth[a, 2] + ev.truth[b, 2])
    assert np.all(np.sign(dydx) == np.sign(sm)) or np.mean(np.sign(dydx) == np.sign(sm)) > 0.99


def test_noise_fraction_and_shuffle():
    ev = tpcgen.pp_event()
    nsig = int((ev.pid >= 0).sum())
    nnoise = ev.n - nsig
    assert nnoise == round(0.05 * nsig)
    # shuffled: noise is not concentrated at the end
    idx = np.nonzero(ev.pid < 0)[0]
    assert idx.mean() < 0.75 * ev.n


@pytest.mark.parametrize("fn", [tpcgen.one_sector_event, tpcgen.pp_event])
def test_efficiency_and_rows(fn):
    ev = fn()
    assert ev.row.max() <= 158 and ev.sector.max() <= 35
    assert np.isfinite(ev.y).all() and np.isfinite(ev.z).all()


def test_pt_spectrum_tail():
    rng = np.random.default_rng(1)
    from tpcgen.events import _pt_exp_tail
    pt = _pt_exp_tail(rng, 200000)
    assert pt.min() >= 0.1 and pt.max() <= 20.0
    # exponential slope below the join: mean of (pT - 0.1) for pT < 1 close to
    # the truncated-exponential value
    assert 0.01 < (pt > 2.0).mean() < 0.06
    assert (pt > 5.0).mean() > 0.0005
