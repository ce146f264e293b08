"""Pins of the multiple-scattering variant (CPU): the generator's kicks
follow the scattering law; the transport's noise terms equal that law
written out independently; fits with the noise model have unit pulls on
scattered tracks, fits without it do not."""
from __future__ import annotations

import numpy as np

import tpcgen
from tpcgen import events as E
import quality as Q

B = -0.00299792458 * 0.5
PACK = [(i, j) for i in range(5) for j in range(i + 1)]


def _law(x0):
    return E.ms_theta2_per_cm(x0), E.PION_MASS ** 2


def test_generator_kicks_follow_the_law():
    """Changes of tan(lambda) between consecutive crossings of a particle,
    divided by theta0 (1 + T^2) of the law for that step, have unit RMS."""
    x0 = 3000.0                      # denser than gas: kicks well above rounding
    ev = E.ms_sector_event(7, 400, x0_cm=x0)
    kk, m2 = _law(x0)
    sig = ev.pid >= 0
    pid, row = ev.pid[sig], ev.row[sig].astype(int)
    tr = ev.truth[sig]
    order = np.lexsort((row, pid))
    pid, row, tr = pid[order], row[order], tr[order]
    X = tpcgen.geometry.row_x().astype(np.float64)
    same = (pid[1:] == pid[:-1]) & (row[1:] == row[:-1] + 1)
    a, b = tr[:-1][same], tr[1:][same]
    T, Qv = a[:, 3], a[:, 4]
    dx = X[row[1:][same]] - X[row[:-1][same]]
    t2 = 1 + T * T
    p = np.sqrt(t2) / np.abs(Qv)
    # path of the step (a close enough chord for the normalisation)
    L = dx * np.sqrt(1 + (a[:, 2] / np.sqrt(1 - a[:, 2] ** 2)) ** 2) * np.sqrt(t2)
    th = np.sqrt(kk * L * (p * p + m2) / p ** 4)
    pull = (b[:, 3] - T) / (th * t2)
    assert len(pull) > 5000
    assert 0.95 < pull.std() < 1.05 and abs(pull.mean()) < 0.05


def test_transport_noise_is_the_law(oracle_lib):
    """Noise added by one transport (zero input covariance): var(s), var(T),
    var(Q), cov(Q, T) equal the law's theta0^2 times (1-s^2)(1+T^2),
    (1+T^2)^2, Q^2 T^2, Q T (1+T^2), theta0^2 from p, beta and the path
    computed directly."""
    rng = np.random.default_rng(3)
    kk, m2 = _law(E.X0_GAS_CM)
    for _ in range(200):
        s, T, q = rng.uniform(-0.6, 0.6), rng.uniform(-1, 1), rng.uniform(-8, 8)
        dx = rng.choice([-1.5, -1.0, 0.75, 1.0])
        ok, p1, C = oracle_lib.predict_ms([0.0, 0.0, s, T, q], np.zeros(15), dx, B, kk, m2)
        assert ok
        s1 = p1[2]
        # exact circle: path length of the step from the turn of the angle
        dphi = np.arcsin(s1) - np.arcsin(s)
        arc = abs(dphi / (B * q)) if abs(B * q) > 1e-12 else abs(dx) * np.sqrt(1 + (s / np.sqrt(1 - s * s)) ** 2)
        t2 = 1 + T * T
        L = arc * np.sqrt(t2)
        pm = np.sqrt(t2) / abs(q)
        th2 = kk * L * (pm * pm + m2) / pm ** 4
        C = dict(zip(PACK, C))
        np.testing.assert_allclose(C[(2, 2)], (1 - s1 * s1) * t2 * th2, rtol=1e-6)
        np.testing.assert_allclose(C[(3, 3)], t2 * t2 * th2, rtol=1e-6)
        np.testing.assert_allclose(C[(4, 4)], q * q * T * T * th2, rtol=1e-6, atol=1e-300)
        np.testing.assert_allclose(C[(4, 3)], q * T * t2 * th2, rtol=1e-6, atol=1e-300)
        for (i, j), v in C.items():
            if (i, j) not in ((2, 2), (3, 3), (4, 4), (4, 3)):
                assert v == 0.0


def _pulls(oracle_lib, x0_fit, seeds, x0_gen):
    P = []
    for k in seeds:
        ev = E.ms_sector_event(1000 + k, 200, x0_cm=x0_gen)
        params = oracle_lib.make_params(x0_cm=x0_fit)
        r = oracle_lib.run_event(ev, precision=32, params=params)
        p, _ = Q.pulls(ev, r.tracks, r.hits)
        P.append(p)
    return np.concatenate(P)


def test_pulls_with_and_without_the_noise_model(oracle_lib):
    """Scattered tracks (X0 = 3000 cm): with the noise model the pulls of
    sin(phi), tan(lambda), q/pT have unit width; without it the angular
    pulls are far too wide."""
    x0 = 3000.0
    with_ms = _pulls(oracle_lib, x0, range(6), x0)
    without = _pulls(oracle_lib, 0.0, range(6), x0)
    assert len(with_ms) > 600
    core = lambda P, i: P[np.abs(P[:, i]) < 6, i]   # noqa: E731
    rms_w = np.array([np.sqrt((core(with_ms, i) ** 2).mean()) for i in range(5)])
    rms_o = np.array([np.sqrt((core(without, i) ** 2).mean()) for i in range(5)])
    assert np.all((rms_w[2:] > 0.85) & (rms_w[2:] < 1.2)), rms_w
    assert rms_o[2] > 1.4 and rms_o[3] > 1.4, rms_o
