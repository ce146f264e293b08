"""Pins of the oracle's float arithmetic and of its double transport written
out independently.

The float path of the oracle takes the tracker's decisions; the GPU is
compared with it bit for bit, so its accuracy needs a check of its own:

* float transport and update against the oracle's double ones, applied to
  the same (float-representable) inputs, on 10^5 random states that include
  |sin phi| close to s_max, tiny and large q/pT and steps of either sign.
  Each output entry's difference is bounded in units of the float unit
  roundoff u = 2^-24 times the magnitude of the terms that entry sums
  (a dropped rounding guard or a quantity formed in a lower precision than
  intended shows up as thousands of units);
* the double transport against a plain numpy transcription of the written
  definition (separate divisions, the mid-angle cosine taken as
  sqrt(1 - s_m^2)), to 1e-12, except dz/dQ, whose leading-order reading
  (mid-angle cosine taken as D/2) is pinned by its exact ratio to the
  definition's value.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

B = -0.00299792458 * 0.5
PACK = [(i, j) for i in range(5) for j in range(i + 1)]
U32 = 2.0 ** -24          # float unit roundoff
N_STATES = 100_000


def unpack(c):
    M = np.zeros((5, 5))
    for k, (i, j) in enumerate(PACK):
        M[i, j] = M[j, i] = c[k]
    return M


def pack(M):
    return np.array([M[i, j] for i, j in PACK])


def random_states(n, seed):
    """States of the kinds a tracklet meets: positions across a sector, all
    directions up to the s_max cut (a fifth of them within 0.05 of it),
    q/pT from 1e-4 (stiff) to 20 c/GeV (loopers), prior-like and narrow
    covariances."""
    rng = np.random.default_rng(seed)
    p = np.zeros((n, 5))
    p[:, 0] = rng.uniform(-40, 40, n)
    p[:, 1] = rng.uniform(-250, 250, n)
    s = rng.uniform(-0.9, 0.9, n)
    edge = rng.uniform(size=n) < 0.2
    s[edge] = np.sign(s[edge]) * rng.uniform(0.9, 0.949, edge.sum())
    p[:, 2] = s
    p[:, 3] = rng.uniform(-1.2, 1.2, n)
    q = np.exp(rng.uniform(np.log(1e-4), np.log(20.0), n)) * rng.choice([-1.0, 1.0], n)
    p[:, 4] = q
    dx = rng.choice([-1.5, -1.0, -0.75, 0.75, 1.0, 1.5], n)
    scale = np.array([0.3, 0.4, 0.03, 0.03, 0.5])
    A = rng.normal(size=(n, 5, 5)) * scale[None, :, None]
    C = A @ A.transpose(0, 2, 1) + np.diag([1e-3, 1e-3, 1e-5, 1e-5, 1e-3])
    # keep the step inside s_max so both precisions transport
    s1 = p[:, 2] + B * p[:, 4] * dx
    ok = np.abs(s1) < 0.949
    p32 = p.astype(np.float32)[ok]
    C32 = np.stack([C[:, i, j] for i, j in PACK], 1).astype(np.float32)[ok]
    return p32, C32, dx.astype(np.float32)[ok], rng


def _steps(oracle_lib, p32, C32, dx, meas=None):
    """Float and double oracle steps on the same inputs (the float values
    converted exactly).  Returns float results, double results, flags."""
    L = oracle_lib.lib()
    n = len(p32)
    pf, Cf = p32.copy(), C32.copy()
    pd, Cd = p32.astype(np.float64), C32.astype(np.float64)
    okf = np.zeros(n, bool)
    okd = np.zeros(n, bool)
    chif = np.zeros(n, np.float32)
    chid = np.zeros(n, np.float64)
    c1f = np.zeros(1, np.float32)
    c1d = np.zeros(1, np.float64)
    for i in range(n):
        a, c = pf[i], Cf[i]
        b, d = pd[i], Cd[i]
        if meas is None:
            okf[i] = L.orc_predict_f(a.ctypes.data, c.ctypes.data, float(dx[i]), float(np.float32(B)), 0.95)
            okd[i] = L.orc_predict_d(b.ctypes.data, d.ctypes.data, float(dx[i]), float(np.float32(B)), 0.95)
        else:
            m = meas[i]
            okf[i] = L.orc_update_f(a.ctypes.data, c.ctypes.data, float(m[0]), float(m[1]), float(m[2]),
                                    float(m[3]), 1e30, 0.999, 0, c1f.ctypes.data)
            okd[i] = L.orc_update_d(b.ctypes.data, d.ctypes.data, float(m[0]), float(m[1]), float(m[2]),
                                    float(m[3]), 1e30, 0.999, 0, c1d.ctypes.data)
            chif[i], chid[i] = c1f[0], c1d[0]
    return pf, Cf, pd, Cd, okf, okd, chif, chid


def _cov_scale(C):
    d = C[:, [0, 2, 5, 9, 14]]
    return np.stack([np.sqrt(d[:, i] * d[:, j]) for i, j in PACK], 1)


def test_float_transport_within_rounding_of_double(oracle_lib):
    """Float transport vs double transport of the same inputs.  Bounds, in
    units of u = 2^-24: y, z, sin phi within 64 u of |x0| + |x1 - x0| (the
    two terms of x1 = x0 + step); T and Q untouched (identical bits);
    covariance entries within 64 u of sqrt(C'_ii C'_jj) (the double
    result's scale: J C J^T of a positive definite C)."""
    p32, C32, dx, _ = random_states(N_STATES, 2026)
    assert len(p32) > 0.95 * N_STATES
    pf, Cf, pd, Cd, okf, okd, _, _ = _steps(oracle_lib, p32, C32, dx)
    assert np.array_equal(okf, okd) and okf.all()
    p0 = p32.astype(np.float64)
    for i in (0, 1, 2):
        scale = np.abs(p0[:, i]) + np.abs(pd[:, i] - p0[:, i])
        err = np.abs(pf[:, i].astype(np.float64) - pd[:, i]) / (U32 * scale)
        assert err.max() <= 64, (i, err.max())
    assert np.array_equal(pf[:, 3:], p32[:, 3:])
    err = np.abs(Cf.astype(np.float64) - Cd) / (U32 * _cov_scale(Cd))
    assert err.max() <= 64, err.max(axis=0)


def _update_term_scales(p0, C0, meas):
    """Magnitudes of the terms each output of the update sums, in double:
    with W = S^-1 and the gains k_i = (C_iy w00 + C_iz w01, C_iy w01 +
    C_iz w11), the i-th parameter sums p_i + k_iy r_y + k_iz r_z and the
    (i, j) covariance entry C_ij - k_iy C_jy - k_iz C_jz; each gain's own
    terms count by magnitude.  W carries the relative error of det S =
    S_yy S_zz - S_yz^2, which cancels by the factor 1 / (1 - rho^2) (rho
    the y-z correlation of S), so the gain terms are weighted by it."""
    vy = meas[:, 2].astype(np.float64)
    vz = meas[:, 3].astype(np.float64)
    s00, s01, s11 = C0[:, 0] + vy, C0[:, 1], C0[:, 2] + vz
    det = s00 * s11 - s01 * s01
    w00, w01, w11 = s11 / det, -s01 / det, s00 / det
    cond = 1.0 / (1.0 - s01 * s01 / (s00 * s11))
    ry = meas[:, 0].astype(np.float64) - p0[:, 0]
    rz = meas[:, 1].astype(np.float64) - p0[:, 1]
    cy = C0[:, [0, 1, 3, 6, 10]]
    cz = C0[:, [1, 2, 4, 7, 11]]
    ky = np.abs(cy * w00[:, None]) + np.abs(cz * w01[:, None])
    kz = np.abs(cy * w01[:, None]) + np.abs(cz * w11[:, None])
    par = np.abs(p0) + cond[:, None] * (ky * np.abs(ry)[:, None] + kz * np.abs(rz)[:, None])
    cov = np.stack([np.abs(C0[:, k]) + cond * (ky[:, i] * np.abs(cy[:, j]) + kz[:, i] * np.abs(cz[:, j]))
                    for k, (i, j) in enumerate(PACK)], 1)
    chi = cond * (np.abs(w00) * ry * ry + 2.0 * np.abs(w01 * ry * rz) + np.abs(w11) * rz * rz)
    return par, cov, chi


def test_float_update_within_rounding_of_double(oracle_lib):
    """Float update vs double update of the same inputs (ungated, so both
    always apply it).  Every parameter, covariance entry and chi2 within
    64 u of the magnitude of the terms it sums (see _update_term_scales)."""
    p32, C32, dx, rng = random_states(N_STATES, 2027)
    n = len(p32)
    meas = np.zeros((n, 4), np.float32)
    meas[:, 0] = p32[:, 0] + rng.normal(size=n).astype(np.float32) * 0.3
    meas[:, 1] = p32[:, 1] + rng.normal(size=n).astype(np.float32) * 0.3
    meas[:, 2] = rng.uniform(0.005, 0.05, n)
    meas[:, 3] = rng.uniform(0.005, 0.05, n)
    pf, Cf, pd, Cd, okf, okd, chif, chid = _steps(oracle_lib, p32, C32, dx, meas)
    p0 = p32.astype(np.float64)
    C0 = C32.astype(np.float64)
    sp, sc, sx = _update_term_scales(p0, C0, meas)
    err = np.abs(pf.astype(np.float64) - pd) / (U32 * sp)
    assert err.max() <= 64, err.max(axis=0)
    err = np.abs(chif.astype(np.float64) - chid) / (U32 * sx)
    assert err.max() <= 64, err.max()
    err = np.abs(Cf.astype(np.float64) - Cd) / (U32 * sc)
    assert err.max() <= 64, err.max(axis=0)


def test_float_gate_decisions_follow_double_away_from_the_cut(oracle_lib):
    """Gated float updates accept exactly where the double ones do, except
    where chi2 lies within rounding (1e-5 relative) of the cut."""
    p32, C32, dx, rng = random_states(20_000, 2028)
    n = len(p32)
    meas = np.zeros((n, 4), np.float32)
    meas[:, 0] = p32[:, 0] + rng.normal(size=n).astype(np.float32) * 2.0
    meas[:, 1] = p32[:, 1] + rng.normal(size=n).astype(np.float32) * 2.0
    meas[:, 2] = rng.uniform(0.005, 0.05, n)
    meas[:, 3] = rng.uniform(0.005, 0.05, n)
    L = oracle_lib.lib()
    accf = np.zeros(n, bool)
    accd = np.zeros(n, bool)
    chi = np.zeros(n)
    c1f = np.zeros(1, np.float32)
    c1d = np.zeros(1, np.float64)
    for i in range(n):
        a, c = p32[i].copy(), C32[i].copy()
        b, d = p32[i].astype(np.float64), C32[i].astype(np.float64)
        m = meas[i]
        accf[i] = L.orc_update_f(a.ctypes.data, c.ctypes.data, float(m[0]), float(m[1]), float(m[2]),
                                 float(m[3]), 16.0, 0.95, 1, c1f.ctypes.data)
        accd[i] = L.orc_update_d(b.ctypes.data, d.ctypes.data, float(m[0]), float(m[1]), float(m[2]),
                                 float(m[3]), 16.0, 0.95, 1, c1d.ctypes.data)
        chi[i] = c1d[0]
    assert 0.2 < accd.mean() < 0.8
    near = np.abs(chi - 16.0) <= 1e-5 * 16.0
    assert np.array_equal(accf[~near], accd[~near])


# ---------------------------------------------------------------------------
# the double transport against the definition written out with numpy

def transport_definition(p, C, dx, b):
    """One row step of the written definition, plainly: separate divisions,
    every quotient formed as written, the mid-angle cosine of dz/dQ as
    sqrt(1 - s_m^2).  Returns (p', J, C' = J C J^T)."""
    y, z, s, T, Q = p
    s1 = s + b * Q * dx
    c0 = np.sqrt(1.0 - s * s)
    c1 = np.sqrt(1.0 - s1 * s1)
    N = s + s1
    D = c0 + c1
    t = N / D
    y1 = y + dx * t
    dl = abs(dx) * np.sqrt(1.0 + t * t)
    u = 0.5 * b * Q * dl
    ds = np.sign(dx) * dl * (1.0 + u * u * (1.0 / 6.0 + u * u * 3.0 / 40.0))
    z1 = z + T * ds
    s_m = N / 2.0
    c_m = np.sqrt(1.0 - s_m * s_m)
    J = np.eye(5)
    J[0, 2] = dx * (2.0 * D + N * (s / c0 + s1 / c1)) / (D * D)
    J[0, 4] = b * dx * dx * (D + N * s1 / c1) / (D * D)
    J[1, 2] = T * dx * N / (c0 * c1 * D)
    J[1, 3] = ds
    J[1, 4] = T * b * s_m * dx * dx / (2.0 * c_m ** 3)
    J[2, 4] = b * dx
    M = unpack(C)
    return np.array([y1, z1, s1, T, Q]), J, J @ M @ J.T


def _oracle_jacobian(oracle_lib, p, dx):
    """Columns s, T, Q of the oracle's Jacobian, read from C' = J C J^T with
    C = e_i e_i^T (J_ii = 1 for these three)."""
    J = np.eye(5)
    for i in (2, 3, 4):
        E = np.zeros((5, 5))
        E[i, i] = 1.0
        ok, _, c = oracle_lib.predict(p, pack(E), dx, B, 0.99)
        assert ok
        J[:, i] = unpack(c)[:, i]
    return J


def test_double_transport_equals_the_definition(oracle_lib):
    """Parameters to 1e-12 of |x0| + |x1 - x0|; every Jacobian entry but
    dz/dQ to 1e-12 of the entry's natural scale; C' to 1e-12 of
    sqrt(C'_ii C'_jj) once dz/dQ is taken as the oracle's (the reading
    pinned in the next test)."""
    rng = np.random.default_rng(31)
    for _ in range(3000):
        s = rng.uniform(-0.9, 0.9)
        T = rng.uniform(-1.2, 1.2)
        Q = np.exp(rng.uniform(np.log(1e-3), np.log(20.0))) * rng.choice([-1.0, 1.0])
        dx = rng.choice([-1.5, -1.0, -0.75, 0.75, 1.0, 1.5])
        if abs(s + B * Q * dx) > 0.94:
            continue
        p = np.array([rng.uniform(-40, 40), rng.uniform(-250, 250), s, T, Q])
        A = rng.normal(size=(5, 5)) * np.array([0.3, 0.4, 0.03, 0.03, 0.5])
        M = A @ A.T + np.diag([1e-3, 1e-3, 1e-5, 1e-5, 1e-3])
        ok, po, co = oracle_lib.predict(p, pack(M), dx, B, 0.99)
        assert ok
        pe, Je, _ = transport_definition(p, pack(M), dx, B)
        scale = np.abs(p) + np.abs(pe - p)
        assert np.all(np.abs(po - pe) <= 1e-12 * np.maximum(scale, 1e-300)), (po, pe)
        Jo = _oracle_jacobian(oracle_lib, np.array([0.0, 0.0, s, T, Q]), dx)
        nat = np.maximum(np.abs(Je), np.abs(dx) * 1e-3)
        d = np.abs(Jo - Je) / nat
        d[1, 4] = 0.0
        assert d.max() <= 1e-12, d
        Jr = Je.copy()
        Jr[1, 4] = Jo[1, 4]
        Ce = Jr @ M @ Jr.T
        err = np.abs(unpack(co) - Ce) / np.sqrt(np.outer(np.diag(Ce), np.diag(Ce)))
        assert err.max() <= 1e-12, err.max()


def test_dz_dq_reading_is_the_exact_mid_angle_ratio(oracle_lib):
    """The oracle's dz/dQ takes the mid-angle cosine as D/2 = (c0 + c1)/2
    instead of the definition's c_m = sqrt(1 - s_m^2), s_m = (s0 + s1)/2.
    With phi_m and delta the half sum and half difference of the two
    angles, D/2 = cos(phi_m) cos(delta) and s_m = sin(phi_m) cos(delta),
    so (D/2)^2 = c_m^2 - sin^2(delta): the ratio of the two readings is
    exactly (c_m^2 / (c_m^2 - sin^2 delta))^(3/2).  Checked to 1e-12.  The
    two readings differ by that ratio minus one, about 1.5 sin^2 delta /
    c_m^2 with sin delta ~ b Q dx / (2 cos phi): below 1e-4 for q/pT under
    1 c/GeV, a few per cent only for looper steps (q/pT ~ 20) near s_max."""
    rng = np.random.default_rng(32)
    worst = 0.0
    for _ in range(3000):
        s = rng.uniform(-0.9, 0.9)
        T = rng.uniform(0.05, 1.2) * rng.choice([-1.0, 1.0])
        Q = np.exp(rng.uniform(np.log(1e-2), np.log(20.0))) * rng.choice([-1.0, 1.0])
        dx = rng.choice([-1.5, -1.0, -0.75, 0.75, 1.0, 1.5])
        s1 = s + B * Q * dx
        if abs(s1) > 0.94:
            continue
        Jo = _oracle_jacobian(oracle_lib, np.array([0.0, 0.0, s, T, Q]), dx)
        _, Je, _ = transport_definition(np.array([0.0, 0.0, s, T, Q]), pack(np.eye(5)), dx, B)
        c_m2 = 1.0 - ((s + s1) / 2.0) ** 2
        sd2 = np.sin((np.arcsin(s1) - np.arcsin(s)) / 2.0) ** 2
        ratio = (c_m2 / (c_m2 - sd2)) ** 1.5
        assert abs(Jo[1, 4] / Je[1, 4] - ratio) <= 1e-12 * ratio
        if abs(Q) < 1.0:
            assert ratio - 1.0 < 1e-4, (s, Q, dx, ratio)
        worst = max(worst, ratio - 1.0)
    assert 0.0 < worst < 0.1, worst
