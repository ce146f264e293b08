"""Pins of the oracle's drift-velocity calibration (CPU).

The beam-axis extrapolation is checked against the exact helices of the
generator (tracks from the origin reach x = 0 at y = 0, z = 0); the fitted
drift error against the value put into the generator; the correction
against its closed-form inverse; the median against numpy's.
"""
from __future__ import annotations

import numpy as np
import pytest

import tpcgen


def test_beam_axis_extrapolation_of_exact_states(oracle_lib):
    """Exact truth states (pT > 0.3; the pp workload has primaries only),
    carried from a cluster's pad row to x = 0, land on the origin to 1e-6 cm."""
    ev = tpcgen.pp_event()
    geo = ev.geometry()
    X = np.asarray(geo["row_x"], np.float32).astype(np.float64)
    pick = (ev.pid >= 0) & (ev.leg == 0) & (ev.row < 30)
    idx = np.nonzero(pick)[0][:400]
    t = np.zeros(len(idx), oracle_lib.TRACK_DTYPE)
    t["par"] = ev.truth[idx]
    t["x_ref"] = X[ev.row[idx]]
    t["sector"] = ev.sector[idx]
    keep = np.abs(t["par"][:, 4]) < 1.0 / 0.3
    y0, z0, ok = oracle_lib.calib_z0(t[keep], geo)
    assert ok.all() and len(y0) > 100
    assert np.abs(y0).max() < 1e-6 and np.abs(z0).max() < 1e-6


@pytest.mark.parametrize("eps", [0.0, 0.004, -0.002])
def test_fit_recovers_the_drift_error(oracle_lib, eps):
    """A drift velocity off by eps in the generator is measured back from
    the tracks to 1e-4 (statistical error of the medians ~2e-5)."""
    ev0 = tpcgen.pbpb_event(tpcgen.seed_for(4, 100), 2000)
    ev = tpcgen.distort_drift(ev0, eps) if eps else ev0
    r = oracle_lib.run_event(ev, precision=32, nthreads=8)
    h = oracle_lib.calib_histogram(r.tracks, ev.geometry())
    assert h.sum() > 2000
    med_a, med_c, e, est = oracle_lib.calib_fit(h, 250.0)
    assert abs(e - eps) < 1e-4, (e, eps)
    assert est == e                 # tracked without correction: the estimate is the measurement
    assert abs(med_a + eps * 250.0) < 0.05 and abs(med_c - eps * 250.0) < 0.05


def test_correction_inverts_the_distortion(oracle_lib):
    ev = tpcgen.pp_event()
    for eps in (0.004, -0.003):
        d = tpcgen.distort_drift(ev, eps)
        zc = oracle_lib.drift_correct(d.sector, d.z, eps, 250.0)
        assert np.abs(zc - ev.z).max() <= 4e-5            # float32 rounding at |z| <= 250


def test_median_is_the_sample_median(oracle_lib):
    """The interpolated histogram median equals numpy's median of the
    selected z0 values to one bin width."""
    ev = tpcgen.distort_drift(tpcgen.pbpb_event(tpcgen.seed_for(4, 102), 2000), 0.003)
    r = oracle_lib.run_event(ev, precision=32, nthreads=8)
    geo = ev.geometry()
    y0, z0, ok = oracle_lib.calib_z0(r.tracks, geo)
    c = oracle_lib.CALIB
    sel = ok & (r.tracks["n_hits"] >= c["n_min"]) & (np.abs(y0) <= c["y0_max"])
    sel &= (z0 >= c["z_lo"]) & (z0 < c["z_hi"])
    h = oracle_lib.calib_histogram(r.tracks, geo)
    assert h.sum() == sel.sum()
    med_a, med_c, _, _ = oracle_lib.calib_fit(h, 250.0)
    w = (c["z_hi"] - c["z_lo"]) / c["n_bins"]
    side = r.tracks["sector"] // 18
    assert abs(med_a - np.median(z0[sel & (side == 0)])) <= w
    assert abs(med_c - np.median(z0[sel & (side == 1)])) <= w


def test_empty_side_gives_nan(oracle_lib):
    h = np.zeros((2, 4000), np.uint32)
    h[0, 2000] = 3
    a, c, e, est = oracle_lib.calib_fit(h, 250.0, eps_tracked=0.001)
    assert a == pytest.approx(0.005, abs=1e-12) and np.isnan(c) and np.isnan(e) and np.isnan(est)


@pytest.mark.parametrize("eps_true,eps_used", [(0.004, 0.0015), (-0.002, 0.001)])
def test_estimate_composes_a_residual_after_correction(oracle_lib, eps_true, eps_used):
    """Events with a drift error eps_true, corrected with a wrong eps_used
    before tracking, leave the residual (eps_true - eps_used) / (1 + eps_used)
    (closed form of correcting z (1 + E) - side E z_max with eps_used); the
    fit measures that residual and its composed estimate gives back eps_true
    to the statistical error of the medians."""
    ev0 = tpcgen.pbpb_event(tpcgen.seed_for(4, 100), 2000)
    d = tpcgen.distort_drift(ev0, eps_true)
    import dataclasses
    ev = dataclasses.replace(d, z=oracle_lib.drift_correct(d.sector, d.z, eps_used, 250.0))
    r = oracle_lib.run_event(ev, precision=32, nthreads=8)
    h = oracle_lib.calib_histogram(r.tracks, ev.geometry())
    _, _, e_r, est = oracle_lib.calib_fit(h, 250.0, eps_tracked=eps_used)
    assert abs(e_r - (eps_true - eps_used) / (1.0 + eps_used)) < 1e-4, e_r
    assert abs(est - eps_true) < 1e-4, est
