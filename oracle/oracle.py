"""Python access to the CPU oracle (test infrastructure only).

The oracle is a plain C++ implementation of the sector tracker, compiled with
g++ (no contraction, no fast-math) into ``oracle/_build/liborc.so``.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may use it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tpc_oracle.cpp")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "liborc.so")

CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
            "-fno-math-errno", "-Wall", "-Wextra", "-Wdouble-promotion", "-Werror",
            "-shared", "-fPIC", "-pthread"]


def build(force: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["g++", *CXXFLAGS, "-o", tmp, SRC], check=True)
        os.replace(tmp, LIB)
    return LIB


class Geometry(ctypes.Structure):
    _fields_ = [("n_sectors", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("row_x", ctypes.c_float * 160), ("bz_tesla", ctypes.c_float),
                ("tan_half_angle", ctypes.c_float), ("z_max", ctypes.c_float),
                ("sigma_y0", ctypes.c_float), ("sigma_y1", ctypes.c_float),
                ("sigma_z0", ctypes.c_float), ("sigma_z1", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("nf_window", ctypes.c_float), ("nf_mmax", ctypes.c_float),
                ("chi2_max", ctypes.c_float), ("k_win", ctypes.c_float),
                ("w_max", ctypes.c_float), ("s_max", ctypes.c_float),
                ("c_s0", ctypes.c_float), ("c_t0", ctypes.c_float), ("c_q0", ctypes.c_float),
                ("m_edge", ctypes.c_float), ("m_z", ctypes.c_float),
                ("n_gap", ctypes.c_int32), ("n_min_tracklet", ctypes.c_int32),
                ("n_min_track", ctypes.c_int32), ("x0_cm", ctypes.c_float),
                ("ms_mass", ctypes.c_float), ("n_min_chain", ctypes.c_int32)]


# The oracle's own constants for the tracker (the values this project
# adopted for a method the paper names without numbers).
class MergeParams(ctypes.Structure):
    _fields_ = [("chi2_max", ctypes.c_float), ("row_gap", ctypes.c_int32),
                ("step_max", ctypes.c_float), ("passes", ctypes.c_int32),
                ("s_max", ctypes.c_float)]


DEFAULT_MERGE = dict(chi2_max=30.0, row_gap=12, step_max=2.0, passes=3, s_max=0.999)

DEFAULT_PARAMS = dict(nf_window=3.0, nf_mmax=16.0, chi2_max=16.0, k_win=4.0, w_max=5.0,
                      s_max=0.95, c_s0=1.0, c_t0=1.0, c_q0=100.0, m_edge=1.0, m_z=1.0,
                      n_gap=6, n_min_tracklet=10, n_min_track=10, x0_cm=0.0, ms_mass=0.13957,
                      n_min_chain=4)

TRACK_DTYPE = np.dtype([("sector", "<i4"), ("n_hits", "<i4"), ("row_in", "<i4"),
                        ("row_out", "<i4"), ("hit_off", "<i8"), ("inner_id", "<i4"),
                        ("start_id", "<i4"), ("x_ref", "<f8"), ("par", "<f8", (5,)),
                        ("cov", "<f8", (15,)), ("chi2", "<f8"), ("ndf", "<i4"),
                        ("tracklet", "<i4")], align=True)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.orc_run.restype = P
        L.orc_run.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Params), ctypes.c_int,
                              ctypes.c_int64, P, P, P, P, ctypes.c_int, ctypes.c_int]
        L.orc_free.argtypes = [P]
        for f in ("orc_n_tracks", "orc_n_track_hits", "orc_n_starts"):
            getattr(L, f).restype = ctypes.c_int64
            getattr(L, f).argtypes = [P]
        L.orc_get_links.argtypes = [P, P, P, P, P]
        L.orc_get_starts.argtypes = [P, P]
        L.orc_get_tracks.argtypes = [P, P, P]
        L.orc_replay_tracks.restype = ctypes.c_int64
        L.orc_replay_tracks.argtypes = [P, P]
        L.orc_n_tracklets.restype = ctypes.c_int64
        L.orc_n_tracklets.argtypes = [P, ctypes.c_int]
        L.orc_get_tracklets.argtypes = [P, ctypes.c_int, P, P, P, P]
        f32, f64 = ctypes.c_float, ctypes.c_double
        L.orc_predict_f.argtypes = [P, P, f32, f32, f32]
        L.orc_predict_d.argtypes = [P, P, f64, f64, f64]
        L.orc_update_f.argtypes = [P, P, f32, f32, f32, f32, f32, f32, ctypes.c_int, P]
        L.orc_predict_ms_d.argtypes = [P, P, f64, f64, f64, f64, f64]
        L.orc_update_d.argtypes = [P, P, f64, f64, f64, f64, f64, f64, ctypes.c_int, P]
        L.orc_kf_steps_f.argtypes = [P, P, P, P, P, ctypes.c_int64, f32, f32, f32]
        L.orc_merge.restype = P
        L.orc_merge.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Params),
                                ctypes.POINTER(MergeParams), P, ctypes.c_int64, P, P, P, P]
        L.orc_merge_free.argtypes = [P]
        for f in ("orc_merge_n_tracks", "orc_merge_n_hits"):
            getattr(L, f).restype = ctypes.c_int64
            getattr(L, f).argtypes = [P]
        L.orc_merge_get.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_rotate_d.argtypes = [P, P, P, f64, f64, f64, f64]
        L.orc_chi2_5.argtypes = [P, P, P]
        L.orc_calib_z0.argtypes = [ctypes.POINTER(Geometry), P, ctypes.c_int64, f64, f64, P, P, P]
        _lib = L
    return _lib


def make_geometry(geo: dict) -> Geometry:
    g = Geometry()
    g.n_sectors = int(geo["n_sectors"])
    g.n_rows = int(geo["n_rows"])
    rx = np.zeros(160, np.float32)
    rx[: g.n_rows] = geo["row_x"]
    for i in range(160):
        g.row_x[i] = float(rx[i])
    for k in ("bz_tesla", "tan_half_angle", "z_max", "sigma_y0", "sigma_y1",
              "sigma_z0", "sigma_z1"):
        setattr(g, k, float(geo[k]))
    return g


def make_params(**over) -> Params:
    d = dict(DEFAULT_PARAMS)
    d.update(over)
    p = Params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class OracleResult:
    precision: int
    up: np.ndarray
    dn: np.ndarray
    upc: np.ndarray
    dnc: np.ndarray
    starts: np.ndarray
    tracks: np.ndarray        # TRACK_DTYPE, canonical order
    hits: np.ndarray          # i32, track hit lists (ascending row)
    replay: np.ndarray | None = None   # TRACK_DTYPE, double replay of a float run
    replay_bad: int = 0
    tracklets: dict | None = None

    def track_hits(self, k: int) -> np.ndarray:
        t = self.tracks[k]
        return self.hits[t["hit_off"]: t["hit_off"] + t["n_hits"]]


def run(sector, row, y, z, geo: dict, precision: int = 32, exhaustive: bool = False,
        nthreads: int = 1, replay: bool = False, tracklet_sectors=(), params=None) -> OracleResult:
    """Track one event on the CPU.  Inputs are the cluster SoA; the cluster
    ID of a cluster is its index."""
    L = lib()
    sector = np.ascontiguousarray(sector, np.uint8)
    row = np.ascontiguousarray(row, np.uint8)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    n = len(y)
    g = make_geometry(geo)
    p = params if params is not None else make_params()
    h = L.orc_run(ctypes.byref(g), ctypes.byref(p), precision, n, _ptr(sector), _ptr(row),
                  _ptr(y), _ptr(z), int(exhaustive), int(nthreads))
    try:
        up, dn, upc, dnc = (np.empty(n, np.int32) for _ in range(4))
        L.orc_get_links(h, _ptr(up), _ptr(dn), _ptr(upc), _ptr(dnc))
        starts = np.empty(L.orc_n_starts(h), np.int32)
        L.orc_get_starts(h, _ptr(starts))
        nt = L.orc_n_tracks(h)
        tracks = np.zeros(nt, TRACK_DTYPE)
        hits = np.empty(L.orc_n_track_hits(h), np.int32)
        L.orc_get_tracks(h, _ptr(tracks), _ptr(hits))
        res = OracleResult(precision, up, dn, upc, dnc, starts, tracks, hits)
        if replay:
            rep = np.zeros(nt, TRACK_DTYPE)
            res.replay_bad = int(L.orc_replay_tracks(h, _ptr(rep)))
            res.replay = rep
        if tracklet_sectors:
            res.tracklets = {}
            for s in tracklet_sectors:
                m = L.orc_n_tracklets(h, s)
                info = np.empty((m, 6), np.int32)
                w = np.empty(m, np.uint32)
                uh = np.empty((m, 159), np.int32)
                dh = np.empty((m, 159), np.int32)
                if m:
                    L.orc_get_tracklets(h, s, _ptr(info), _ptr(w), _ptr(uh), _ptr(dh))
                res.tracklets[s] = dict(start=info[:, 0], n=info[:, 1], row_in=info[:, 2],
                                        row_out=info[:, 3], valid=info[:, 4].astype(bool),
                                        r0=info[:, 5], weight=w, uhit=uh, dhit=dh)
        return res
    finally:
        L.orc_free(h)


def run_event(ev, **kw) -> OracleResult:
    return run(ev.sector, ev.row, ev.y, ev.z, ev.geometry(), **kw)


# ---- single Kalman steps ----------------------------------------------------

def predict(p, C, dx, b, smax=0.95, precision=64):
    dt = np.float64 if precision == 64 else np.float32
    p = np.array(p, dt)
    C = np.array(C, dt)
    f = lib().orc_predict_d if precision == 64 else lib().orc_predict_f
    ok = f(_ptr(p), _ptr(C), dx, b, smax)
    return bool(ok), p, C


def predict_ms(p, C, dx, b, kk, m2, smax=0.95):
    """Double transport with the scattering noise (kk = k^2/X0, m2 = mass^2)."""
    p = np.array(p, np.float64)
    C = np.array(C, np.float64)
    ok = lib().orc_predict_ms_d(_ptr(p), _ptr(C), dx, b, smax, kk, m2)
    return bool(ok), p, C


def update(p, C, my, mz, vy, vz, chi2max=16.0, smax=0.95, gated=True, precision=64):
    dt = np.float64 if precision == 64 else np.float32
    p = np.array(p, dt)
    C = np.array(C, dt)
    chi2 = np.zeros(1, dt)
    f = lib().orc_update_d if precision == 64 else lib().orc_update_f
    ok = f(_ptr(p), _ptr(C), my, mz, vy, vz, chi2max, smax, int(gated), _ptr(chi2))
    return bool(ok), p, C, float(chi2[0])


def kf_steps_f32(state, dx, meas, b, smax=0.95, chi2max=16.0):
    """Float transport + gated update of n states (state[n, 20] = p, C;
    meas[n, 4] = y, z, var_y, var_z).  Returns (state', bits, chi2); bits =
    transport ok | accepted << 1, chi2 as computed by the update."""
    st = np.ascontiguousarray(state, np.float32).copy()
    dx = np.ascontiguousarray(dx, np.float32)
    meas = np.ascontiguousarray(meas, np.float32)
    n = len(st)
    bits = np.zeros(n, np.int32)
    chi2 = np.zeros(n, np.float32)
    lib().orc_kf_steps_f(_ptr(st), _ptr(dx), _ptr(meas), _ptr(bits), _ptr(chi2), n, b, smax, chi2max)
    return st, bits, chi2


def curvature_b(bz_tesla: float) -> float:
    """b = -c Bz in cm^-1 per (c/GeV); d(phi)/dl = b * q/pT."""
    return -0.00299792458 * float(bz_tesla)


# ---- cross-sector merger ------------------------------------------------------

@dataclass
class MergeResult:
    tracks: np.ndarray        # TRACK_DTYPE, canonical order (merged and single)
    hits: np.ndarray
    n_segments: np.ndarray    # per output track
    link_out: np.ndarray      # per input track: linked outer segment or -1
    best_out: np.ndarray      # per input track: best outer candidate or -1
    best_chi2: np.ndarray
    merged_into: np.ndarray   # per input track: output track index

    def track_hits(self, k: int) -> np.ndarray:
        t = self.tracks[k]
        return self.hits[t["hit_off"]: t["hit_off"] + t["n_hits"]]


def merge(tracks, hits, row, y, z, geo: dict, params=None, **over) -> MergeResult:
    """Join the track segments of one event across sector boundaries (input:
    the tracks of `run` for that event, canonical order)."""
    L = lib()
    tracks = np.ascontiguousarray(tracks, TRACK_DTYPE)
    hits = np.ascontiguousarray(hits, np.int32)
    row = np.ascontiguousarray(row, np.uint8)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    g = make_geometry(geo)
    p = params if params is not None else make_params()
    m = MergeParams()
    d = dict(DEFAULT_MERGE)
    d.update(over)
    for k, v in d.items():
        setattr(m, k, v)
    n = len(tracks)
    h = L.orc_merge(ctypes.byref(g), ctypes.byref(p), ctypes.byref(m), _ptr(tracks), n,
                    _ptr(hits), _ptr(row), _ptr(y), _ptr(z))
    try:
        nt = L.orc_merge_n_tracks(h)
        out = np.zeros(nt, TRACK_DTYPE)
        oh = np.empty(L.orc_merge_n_hits(h), np.int32)
        nseg = np.empty(nt, np.int32)
        lo, bo, mi = (np.empty(n, np.int32) for _ in range(3))
        bc = np.empty(n, np.float64)
        L.orc_merge_get(h, _ptr(out), _ptr(oh), _ptr(nseg), _ptr(lo), _ptr(bo), _ptr(bc), _ptr(mi))
        return MergeResult(out, oh, nseg, lo, bo, bc, mi)
    finally:
        L.orc_merge_free(h)


def rotate(p, C, x, ca, sa, b, smax=0.95):
    p = np.array(p, np.float64)
    C = np.array(C, np.float64)
    xx = np.array([x], np.float64)
    ok = lib().orc_rotate_d(_ptr(p), _ptr(C), _ptr(xx), ca, sa, b, smax)
    return bool(ok), p, C, float(xx[0])


def chi2_5(S, d):
    S = np.ascontiguousarray(S, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros(1, np.float64)
    ok = lib().orc_chi2_5(_ptr(S), _ptr(d), _ptr(out))
    return bool(ok), float(out[0])


# ---- drift-velocity calibration -------------------------------------------------
# Accumulate, per side (sectors 0-17: A, z > 0; 18-35: C), the beam-axis z0 of
# primary-like tracks into an integer histogram; the fit takes each side's
# median (linear inside the median bin) and eps = (med_C - med_A) / (2 z_max).

CALIB = dict(n_bins=4000, z_lo=-20.0, z_hi=20.0, n_min=30, y0_max=2.0, step_max=2.0,
             s_max=0.999)


def calib_z0(tracks, geo: dict):
    """(y0, z0, ok) per track: parameters transported to x = 0."""
    tracks = np.ascontiguousarray(tracks, TRACK_DTYPE)
    n = len(tracks)
    y0, z0 = np.zeros(n), np.zeros(n)
    ok = np.zeros(n, np.int32)
    g = make_geometry(geo)
    lib().orc_calib_z0(ctypes.byref(g), _ptr(tracks), n, CALIB["step_max"], CALIB["s_max"],
                       _ptr(y0), _ptr(z0), _ptr(ok))
    return y0, z0, ok.astype(bool)


def calib_histogram(tracks, geo: dict, n_bins=None, z_lo=None, z_hi=None):
    """[2, n_bins] uint32 counts of z0 for the selected tracks of one event."""
    n_bins = n_bins or CALIB["n_bins"]
    z_lo = CALIB["z_lo"] if z_lo is None else z_lo
    z_hi = CALIB["z_hi"] if z_hi is None else z_hi
    y0, z0, ok = calib_z0(tracks, geo)
    w = (float(np.float32(z_hi)) - float(np.float32(z_lo))) / n_bins
    lo = float(np.float32(z_lo))
    sel = ok & (tracks["n_hits"] >= CALIB["n_min"]) & (np.abs(y0) <= CALIB["y0_max"])
    f = (z0 - lo) / w
    sel &= (f >= 0.0) & (f < n_bins)
    b = np.floor(f[sel]).astype(np.int64)
    side = (np.asarray(tracks["sector"])[sel] // 18).astype(np.int64)
    h = np.zeros((2, n_bins), np.uint32)
    np.add.at(h, (side, b), 1)
    return h


def calib_fit(hist, z_max: float, z_lo=None, z_hi=None, eps_tracked: float = 0.0):
    """(median z0 of side A, of side C, eps_r, E); NaN where a side is empty.
    eps_r is the drift error measured on the histogram's events; they were
    tracked after a correction with eps_tracked, which leaves the error
    eps_r = (E - eps_tracked) / (1 + eps_tracked) of a true error E, so the
    estimate to adopt is E = eps_tracked + eps_r (1 + eps_tracked)."""
    n_bins = hist.shape[1]
    z_lo = CALIB["z_lo"] if z_lo is None else z_lo
    z_hi = CALIB["z_hi"] if z_hi is None else z_hi
    lo = float(np.float32(z_lo))
    w = (float(np.float32(z_hi)) - lo) / n_bins
    med = []
    for side in range(2):
        c = hist[side].astype(np.int64)
        n = int(c.sum())
        if n == 0:
            med.append(float("nan"))
            continue
        half = n / 2.0
        cum = np.concatenate([[0], np.cumsum(c)])
        b = int(np.nonzero(cum[1:] >= half)[0][0])
        med.append(lo + (b + (half - float(cum[b])) / float(c[b])) * w)
    zm = float(np.float32(z_max))
    eps_r = (med[1] - med[0]) / (2.0 * zm)
    return med[0], med[1], eps_r, eps_tracked + eps_r * (1.0 + eps_tracked)


def drift_correct(sector, z, eps: float, z_max: float):
    """Cluster z corrected for a drift-velocity error eps (float32 out)."""
    s = np.where(np.asarray(sector) < 18, 1.0, -1.0)
    zm = float(np.float32(z_max))
    return ((np.asarray(z, np.float64) + s * eps * zm) / (1.0 + eps)).astype(np.float32)
