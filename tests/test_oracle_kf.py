"""Pins of the oracle's Kalman-filter arithmetic against closed forms,
finite differences, the textbook dense Kalman update, least squares and
generator truth.  A dropped term, a sign, an index or a transposed operand in
the transport, the Jacobian or the update fails at least one of these."""
import numpy as np
import pytest

import tpcgen
from tpcgen import geometry as G
import quality as Q

B = -0.00299792458 * 0.5
PACK = [(i, j) for i in range(5) for j in range(i + 1)]


def unpack(c):
    M = np.zeros((5, 5))
    for k, (i, j) in enumerate(PACK):
        M[i, j] = M[j, i] = c[k]
    return M


def pack(M):
    return np.array([M[i, j] for i, j in PACK])


# ---------------------------------------------------------------------------
# transport
# ---------------------------------------------------------------------------

def _consecutive_truth(ev):
    """(state at row r, state at row r+1, dx) for outgoing legs of the same
    particle in the same sector."""
    sig = np.nonzero((ev.pid >= 0) & (ev.leg == 0))[0]
    key = ev.pid[sig].astype(np.int64) * 1000 + ev.sector[sig].astype(np.int64) * 200 + ev.row[sig]
    order = np.argsort(key)
    s, k = sig[order], key[order]
    nxt = np.nonzero(np.diff(k) == 1)[0]
    a, b = s[nxt], s[nxt + 1]
    x = G.row_x().astype(np.float64)
    return ev.truth[a], ev.truth[b], x[ev.row[b]] - x[ev.row[a]]


@pytest.mark.parametrize("reverse", [False, True])
def test_transport_matches_exact_helix(oracle_lib, reverse):
    """Predicting the true state from one pad row to the next lands on the
    generator's exact helix crossing (closed form, trigonometric)."""
    ev = tpcgen.one_sector_event()
    s0, s1, dx = _consecutive_truth(ev)
    if reverse:
        s0, s1, dx = s1, s0, -dx
    idx = np.random.default_rng(0).choice(len(dx), 3000, replace=False)
    C = pack(np.eye(5))
    for i in idx:
        ok, p, _ = oracle_lib.predict(s0[i], C, dx[i], B, 0.99)
        assert ok
        assert abs(p[0] - s1[i, 0]) < 1e-9
        assert abs(p[1] - s1[i, 1]) < 1e-9 * max(1.0, abs(s1[i, 1]))
        assert abs(p[2] - s1[i, 2]) < 1e-12
        assert p[3] == s0[i, 3] and p[4] == s0[i, 4]


def test_transport_arc_length_series(oracle_lib):
    """z advances by T times the exact arc 2R asin(chord / 2R); the series in
    the transport is within 1e-9 relative for |u| <= 0.05."""
    rng = np.random.default_rng(3)
    for _ in range(500):
        q = rng.uniform(-10, 10)
        s = rng.uniform(-0.6, 0.6)
        dx = rng.choice([-1.5, -1.0, -0.75, 0.75, 1.0, 1.5]) * rng.uniform(0.5, 3.0)
        s1 = s + B * q * dx
        if abs(s1) > 0.9:
            continue
        ok, p, _ = oracle_lib.predict([0.0, 0.0, s, 1.0, q], pack(np.eye(5)), dx, B, 0.95)
        assert ok
        # exact: arc = (asin(s1) - asin(s)) / (B q)
        arc = (np.arcsin(s1) - np.arcsin(s)) / (B * q) if q != 0 else dx / np.sqrt(1 - s * s)
        chord = np.hypot(dx, p[0])
        u = 0.5 * abs(B * q) * chord
        if u <= 0.05:
            assert abs(p[1] - arc) <= 1e-9 * abs(arc)
        # y: exact circle
        y_exact = (np.sqrt(1 - s * s) - np.sqrt(1 - s1 * s1)) / (B * q) if q != 0 else dx * s / np.sqrt(1 - s * s)
        assert abs(p[0] - y_exact) < 1e-10 * max(1, abs(y_exact))


def test_transport_refuses_beyond_smax(oracle_lib):
    ok, p, C = oracle_lib.predict([1.0, 2.0, 0.94, 0.1, 20.0], pack(np.eye(5)), 1.5, B, 0.95)
    assert (0.94 + B * 20.0 * 1.5) < 0.95
    assert ok
    ok, p2, _ = oracle_lib.predict([1.0, 2.0, 0.94, 0.1, -20.0], pack(np.eye(5)), 1.5, B, 0.95)
    assert not ok
    assert np.array_equal(p2, [1.0, 2.0, 0.94, 0.1, -20.0])


# ---------------------------------------------------------------------------
# Jacobian
# ---------------------------------------------------------------------------

def _jac_columns(oracle_lib, p, dx):
    """Columns s, T, Q of the transport Jacobian read from C' = J C J^T with
    C = e_i e_i^T (J_ii = 1 for those three)."""
    J = np.eye(5)
    for i in (2, 3, 4):
        E = np.zeros((5, 5))
        E[i, i] = 1.0
        ok, _, c = oracle_lib.predict(p, pack(E), dx, B, 0.99)
        assert ok
        J[:, i] = unpack(c)[:, i]
    return J


def test_jacobian_vs_finite_differences(oracle_lib):
    rng = np.random.default_rng(11)
    worst = np.zeros((5, 5))
    for _ in range(300):
        # the Jacobian does not depend on (y, z); zero them so the central
        # differences are not swamped by round-off of large coordinates
        p = np.array([0.0, 0.0, rng.uniform(-0.7, 0.7), rng.uniform(-1.2, 1.2), rng.uniform(-6, 6)])
        dx = rng.choice([-1.5, -1.0, -0.75, 0.75, 1.0, 1.5])
        J = _jac_columns(oracle_lib, p, dx)
        Jfd = np.eye(5)
        for i, h in ((2, 1e-5), (3, 1e-5), (4, 1e-4)):
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            _, a, _ = oracle_lib.predict(pp, pack(np.eye(5)), dx, B, 0.99)
            _, b, _ = oracle_lib.predict(pm, pack(np.eye(5)), dx, B, 0.99)
            Jfd[:, i] = (a - b) / (2 * h)
        scale = np.maximum(np.abs(Jfd), 1e-6)
        worst = np.maximum(worst, np.abs(J - Jfd) / scale)
    worst[1, 4] = 0.0      # dz/dQ is kept to leading order: pinned below
    assert worst.max() < 1e-6, worst


def test_jacobian_dz_dq_leading_order(oracle_lib):
    """dz/dQ against its exact closed form T (dx/c1 - arc)/Q (arc =
    (asin s1 - asin s)/(bQ)): the leading-order entry is within 1% of its
    natural scale |T b| dx^2 (a wrong sign or factor is off by ~100%)."""
    rng = np.random.default_rng(12)
    for _ in range(2000):
        s, tl, q = rng.uniform(-0.7, 0.7), rng.uniform(-1.2, 1.2), rng.uniform(-6, 6)
        dx = rng.choice([-1.5, -1.0, -0.75, 0.75, 1.0, 1.5])
        J = _jac_columns(oracle_lib, np.array([0.0, 0.0, s, tl, q]), dx)
        s1 = s + B * q * dx
        arc = (np.arcsin(s1) - np.arcsin(s)) / (B * q)
        exact = tl * (dx / np.sqrt(1 - s1 * s1) - arc) / q
        assert abs(J[1, 4] - exact) <= 1e-2 * abs(tl * B) * dx * dx


# ---------------------------------------------------------------------------
# update
# ---------------------------------------------------------------------------

def _random_spd(rng):
    A = rng.normal(size=(5, 5)) * np.array([0.3, 0.5, 0.05, 0.05, 1.0])
    return A @ A.T + np.diag([0.01, 0.02, 1e-4, 1e-4, 0.01])


def test_update_matches_textbook_kalman(oracle_lib):
    """Against the dense form: K = C H^T (H C H^T + R)^-1, p' = p + K r,
    C' = (I - K H) C, chi2 = r^T S^-1 r."""
    rng = np.random.default_rng(5)
    H = np.zeros((2, 5))
    H[0, 0] = H[1, 1] = 1.0
    for _ in range(500):
        C = _random_spd(rng)
        p = rng.normal(size=5)
        m = p[:2] + rng.normal(size=2) * 0.3
        vy, vz = rng.uniform(0.005, 0.05, 2)
        Rm = np.diag([vy, vz])
        S = H @ C @ H.T + Rm
        K = C @ H.T @ np.linalg.inv(S)
        r = m - H @ p
        pe = p + K @ r
        Ce = (np.eye(5) - K @ H) @ C
        chi2e = r @ np.linalg.solve(S, r)
        ok, pn, cn, chi2 = oracle_lib.update(p, pack(C), m[0], m[1], vy, vz, gated=False)
        assert ok
        assert np.allclose(pn, pe, rtol=1e-12, atol=1e-12 * np.abs(pe).max())
        assert np.allclose(unpack(cn), Ce, rtol=1e-10, atol=1e-12 * np.abs(Ce).max())
        assert abs(chi2 - chi2e) <= 1e-10 * max(1.0, chi2e)


def test_update_gate(oracle_lib):
    C = pack(np.diag([0.01, 0.01, 1e-3, 1e-3, 0.1]))
    p = [0.0, 0.0, 0.1, 0.2, 1.0]
    # 1 cm residual with S = 0.02 -> chi2 = 50 > 16: refused, state unchanged
    ok, pn, cn, chi2 = oracle_lib.update(p, C, 1.0, 0.0, 0.01, 0.01, chi2max=16.0, gated=True)
    assert not ok and np.isclose(chi2, 50.0)
    assert np.array_equal(pn, p) and np.array_equal(cn, C)
    ok, pn, cn, chi2 = oracle_lib.update(p, C, 0.1, 0.0, 0.01, 0.01, chi2max=16.0, gated=True)
    assert ok and np.isclose(chi2, 0.5) and np.isclose(pn[0], 0.05)


# ---------------------------------------------------------------------------
# fits
# ---------------------------------------------------------------------------

def test_noiseless_fit_equals_truth(oracle_lib):
    """Unsmeared clusters with the same error model: the refitted state at the
    innermost hit is the truth to within 1e-3 sigma."""
    ev = tpcgen.tiny_event(21, n_tracks=5, smear=False)
    r = oracle_lib.run_event(ev, precision=64)
    assert len(r.tracks) == 5
    for t in r.tracks:
        tr = ev.truth[t["inner_id"]]
        sig = np.sqrt(np.array(t["cov"])[[0, 2, 5, 9, 14]])
        assert np.all(np.abs(np.array(t["par"]) - tr) <= 1e-3 * sig), (t["par"], tr, sig)


def test_straight_tracks_match_least_squares(oracle_lib):
    """B_z = 0: the fit is a straight line; it equals the weighted least
    squares line y(x), z(path) to 3e-2 sigma in the parameters and 1e-2 in
    the errors (the extended filter linearises tan(phi) at its running
    estimate, which leaves a ~1e-2 sigma difference to the exact optimum)."""
    from scipy.optimize import least_squares
    rng = np.random.default_rng(9)
    x = G.row_x().astype(np.float64)
    sy, sz = 0.1, 0.15
    ids = []
    Y, Z, R = [], [], []
    truth = []
    for k in range(4):
        phi = np.deg2rad(-6 + 4 * k)
        T = 0.2 + 0.15 * k
        y = x * np.tan(phi)
        z = T * x / np.cos(phi)
        Y.append(y + rng.normal(size=159) * sy)
        Z.append(z + rng.normal(size=159) * sz)
        R.append(np.arange(159))
        truth.append((phi, T))
    y = np.concatenate(Y).astype(np.float32)
    z = np.concatenate(Z).astype(np.float32)
    row = np.concatenate(R).astype(np.uint8)
    sec = np.zeros(len(y), np.uint8)
    geo = G.geometry_dict((sy, 0.0, sz, 0.0))
    geo["bz_tesla"] = np.float32(0.0)
    r = oracle_lib.run(sec, row, y, z, geo, precision=64)
    assert len(r.tracks) == 4
    for k in range(4):
        t = r.tracks[k]
        h = r.track_hits(k)
        xr = x[row[h]].astype(np.float64)
        x0 = t["x_ref"]
        yy, zz = y[h].astype(np.float64), z[h].astype(np.float64)

        def res(q):
            y0, s, z0, T = q
            c = np.sqrt(1 - s * s)
            return np.concatenate([(y0 + (xr - x0) * s / c - yy) / sy,
                                   (z0 + T * (xr - x0) / c - zz) / sz])
        q0 = np.array(t["par"])[[0, 2, 1, 3]]
        sol = least_squares(res, q0, xtol=1e-15, ftol=1e-15, gtol=1e-15)
        Jm = sol.jac
        cov = np.linalg.inv(Jm.T @ Jm)
        lsq = sol.x
        par = np.array(t["par"])[[0, 2, 1, 3]]
        C = unpack(t["cov"])[np.ix_([0, 2, 1, 3], [0, 2, 1, 3])]
        sig = np.sqrt(np.diag(cov))
        assert np.all(np.abs(par - lsq) <= 3e-2 * sig), (par, lsq, sig)
        assert np.allclose(np.sqrt(np.diag(C)), sig, rtol=1e-2)


def test_pulls_and_chi2_one_sector(oracle_lib):
    """Generator truth: pulls of the 5 parameters at the innermost hit have
    unit width and zero mean, chi2/ndf averages 1 (float decisions, 20
    events of the one-sector workload)."""
    P, C2 = [], []
    for k in range(1, 21):
        ev = tpcgen.one_sector_event(tpcgen.seed_for(0) + k)
        r = oracle_lib.run_event(ev, precision=32)
        p, c2 = Q.pulls(ev, r.tracks, r.hits)
        P.append(p)
        C2.append(c2)
    P = np.concatenate(P)
    C2 = np.concatenate(C2)
    assert len(P) > 2000
    rms = np.sqrt((P ** 2).mean(0))
    assert np.all((rms > 0.9) & (rms < 1.1)), rms
    assert np.all(np.abs(P.mean(0)) < 0.1), P.mean(0)
    assert 0.9 < C2.mean() < 1.1


def test_pulls_pbpb_with_loopers_and_secondaries(oracle_lib):
    """Pulls stay unit-width on a Pb-Pb-shaped event (secondaries, looper
    legs followed in either direction); a few mixed tracks aside, the
    central 98% of each pull lies within +-4."""
    ev = tpcgen.pbpb_event(tpcgen.seed_for(2) + 5, 3000)
    r = oracle_lib.run_event(ev, precision=32, nthreads=8)
    p, c2 = Q.pulls(ev, r.tracks, r.hits)
    assert len(p) > 5000
    lo, hi = np.percentile(p, [1, 99], axis=0)
    assert np.all(lo > -4) and np.all(hi < 4), (lo, hi)
    core = np.abs(p) < 5
    rms = np.sqrt([(p[core[:, i], i] ** 2).mean() for i in range(5)])
    assert np.all((rms > 0.85) & (rms < 1.2)), rms
    assert 0.85 < np.median(c2) < 1.15


@pytest.mark.parametrize("make", [tpcgen.one_sector_event, tpcgen.pp_event])
def test_float_run_matches_double_replay(oracle_lib, make):
    """The float run's track parameters and covariances equal the double
    replay of the same decisions: 1e-4 relative (floors 10 cm, 10 cm, 0.1,
    0.1, 0.1) and 1e-3 of sqrt(C_ii C_jj)."""
    ev = make()
    r = oracle_lib.run_event(ev, precision=32, replay=True)
    assert r.replay_bad == 0
    f, d = r.tracks, r.replay
    floor = np.array([10.0, 10.0, 0.1, 0.1, 0.1])
    pe = np.abs(f["par"] - d["par"]) / np.maximum(np.abs(d["par"]), floor)
    assert pe.max() <= 1e-4
    diag = d["cov"][:, [0, 2, 5, 9, 14]]
    den = np.stack([np.sqrt(diag[:, i] * diag[:, j]) for i, j in PACK], 1)
    assert (np.abs(f["cov"] - d["cov"]) / den).max() <= 1e-3
