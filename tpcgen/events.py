"""Seeded synthetic TPC events (stand-ins for the ALICE Pb-Pb / pp data the
paper's tracker ran on; the paper's own events are not available).

Particles are exact helices in a uniform field B_z (no material, no multiple
scattering, no energy loss).  Every crossing of a pad-row plane inside a
sector's acceptance becomes one cluster, smeared with the stated Gaussian
errors; a fraction of uniformly distributed noise clusters is added and the
cluster list is shuffled, so the cluster ID (input index) carries no order.

Per cluster the generator also records the truth: particle index (-1 for
noise), the (sector, leg) it belongs to and the exact local track state at the
crossing, written as the tracker sees the leg when it follows it towards
larger x (a returning looper leg shows up with sin phi, T and Q negated).

Nothing here is tracker arithmetic: the generator uses trigonometry on the
global helix, while the tracker propagates a local state row by row.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import geometry as G

SEED_BASE = 1712094160

# config names, in the order of the workloads they describe
CFG_ONE_SECTOR = 0      # one sector, 200 tracks
CFG_PP = 1              # 36 sectors, 60 primaries
CFG_CENTRAL = 2         # 36 sectors, 15000 primaries + secondaries + loopers
CFG_BATCH = 3           # 64 events of the central shape, multiplicity 50..15000
CFG_SERVE = 4           # Poisson mix of pp / peripheral / central


@dataclass
class Event:
    name: str
    seed: int
    sector: np.ndarray      # u8[N]
    row: np.ndarray         # u8[N]
    y: np.ndarray           # f32[N]
    z: np.ndarray           # f32[N]
    q: np.ndarray           # f32[N] (charge; carried, unused by tracking)
    pid: np.ndarray         # i32[N], -1 = noise
    leg: np.ndarray         # i32[N], -1 = noise
    truth: np.ndarray       # f64[N, 5] local (y, z, sin phi, tan lambda, q/pT), NaN for noise
    sigma: tuple            # (sy0, sy1, sz0, sz1)
    particles: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.y.shape[0])

    def geometry(self) -> dict:
        return G.geometry_dict(self.sigma)


# ----------------------------------------------------------------------------
# particle spectra
# ----------------------------------------------------------------------------

def _pt_loguniform(rng, n, lo, hi):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def _pt_exp(rng, n, slope=0.5, lo=0.1):
    return lo + rng.exponential(slope, n)


def _pt_exp_tail(rng, n, slope=0.5, lo=0.1, pj=2.0, hi=20.0, power=4.0):
    """pdf ~ exp(-pT/slope) on [lo, pj), joined continuously to
    exp(-pj/slope) * (pT/pj)^-power on [pj, hi] (a power-law tail)."""
    w_exp = slope * (np.exp(-lo / slope) - np.exp(-pj / slope))
    a = np.exp(-pj / slope)
    w_tail = a * pj / (power - 1.0) * (1.0 - (hi / pj) ** (1.0 - power))
    out = np.empty(n)
    is_tail = rng.uniform(size=n) < w_tail / (w_exp + w_tail)
    nt = int(is_tail.sum())
    ne = n - nt
    # exponential part by inversion on [lo, pj)
    u = rng.uniform(size=ne)
    e0, e1 = np.exp(-lo / slope), np.exp(-pj / slope)
    out[~is_tail] = -slope * np.log(e0 - u * (e0 - e1))
    # power-law part by inversion on [pj, hi]
    u = rng.uniform(size=nt)
    k = 1.0 - power
    out[is_tail] = pj * (1.0 + u * ((hi / pj) ** k - 1.0)) ** (1.0 / k)
    return out


def _particles(rng, n, pt, phi_lo, phi_hi, eta_lo, eta_hi, kind,
               vertex_radius=None):
    """Particle table: vertex (vx, vy, vz), pT, phi0, eta, charge, kind."""
    phi = rng.uniform(phi_lo, phi_hi, n)
    eta = rng.uniform(eta_lo, eta_hi, n)
    charge = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    vx = np.zeros(n)
    vy = np.zeros(n)
    vz = np.zeros(n)
    if vertex_radius is not None:
        r = rng.uniform(0.0, vertex_radius, n)
        a = rng.uniform(0.0, 2 * np.pi, n)
        eta_v = rng.uniform(-0.9, 0.9, n)
        vx, vy, vz = r * np.cos(a), r * np.sin(a), r * np.sinh(eta_v)
        phi = a + rng.uniform(-0.5, 0.5, n)
    return dict(vx=vx, vy=vy, vz=vz, pt=pt, phi=phi, eta=eta, charge=charge,
                kind=np.full(n, kind, dtype=np.int8))


def _concat(parts):
    keys = parts[0].keys()
    return {k: np.concatenate([p[k] for p in parts]) for k in keys}


# ----------------------------------------------------------------------------
# helix / pad-row-plane crossings
# ----------------------------------------------------------------------------

def _sector_candidates(p, xc, yc, hR, l_max):
    """Azimuthal sector indices (0..17) each particle can reach inside the
    TPC: sample the path, take the sectors of samples at radius >= 70 cm and
    their neighbours.  Returns (particle index, azimuth sector) pairs."""
    ns = 96
    t = np.linspace(0.0, 1.0, ns)[None, :] * l_max[:, None]        # arc length
    R = np.abs(hR)[:, None]
    phi = p["phi"][:, None] + np.sign(hR)[:, None] * t / R
    X = xc[:, None] + hR[:, None] * np.sin(phi)
    Y = yc[:, None] - hR[:, None] * np.cos(phi)
    rad = np.hypot(X, Y)
    az = np.mod(np.arctan2(Y, X), 2 * np.pi)
    sec = np.floor(az / np.deg2rad(20.0)).astype(np.int64) % 18
    ok = rad >= 70.0
    hit = np.zeros((len(l_max), 18), dtype=bool)
    ip = np.broadcast_to(np.arange(len(l_max))[:, None], sec.shape)
    for d in (-1, 0, 1):
        hit[ip[ok], (sec[ok] + d) % 18] = True
    return np.nonzero(hit)


def _crossings(p, sectors_allowed, x_rows):
    """All (particle, sector, row) crossings inside the acceptance.

    Returns dict of flat arrays: pid, sector, row, y, z (true local), s, T, Q
    (outward-seen truth), leg.
    """
    npart = len(p["pt"])
    R = p["pt"] / (G.C_LIGHT * G.BZ_TESLA)            # radius, cm
    h = -np.sign(p["charge"] * G.BZ_TESLA)            # d(phi)/dl = h / R
    hR = h * R
    phi0 = p["phi"]
    xc = p["vx"] - hR * np.sin(phi0)
    yc = p["vy"] + hR * np.cos(phi0)
    T = np.sinh(p["eta"])
    Q = p["charge"] / p["pt"]

    # arc length at which the particle leaves the drift volume
    l_turns = 2.0 * 2.0 * np.pi * R                     # at most two turns
    rho = np.hypot(xc, yc)
    psi = np.arctan2(yc, xc)
    A = rho ** 2 + R ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        w = (G.R_EXIT ** 2 - A) / (2.0 * hR * rho)
    l_r = np.full(npart, np.inf)
    can_exit = np.abs(w) <= 1.0
    aw = np.arcsin(np.clip(w, -1.0, 1.0))
    for sol in (psi + aw, psi + np.pi - aw):
        th = np.mod(h * (sol - phi0), 2 * np.pi)
        l_r = np.where(can_exit, np.minimum(l_r, R * th), l_r)
    with np.errstate(divide="ignore", invalid="ignore"):
        l_z = np.where(T != 0, (np.sign(T) * G.Z_MAX - p["vz"]) / T, np.inf)
    l_max = np.minimum(np.minimum(l_turns, l_r), l_z)

    ip, ia = _sector_candidates(p, xc, yc, hR, l_max)
    alpha = G.sector_alpha(ia)
    ca, sa = np.cos(alpha), np.sin(alpha)
    xr = x_rows.astype(np.float64)[None, :]                      # [1, 159]
    nC = (xc[ip] * ca + yc[ip] * sa)[:, None]
    yC = (-xc[ip] * sa + yc[ip] * ca)[:, None]
    hRp = hR[ip][:, None]
    v = (xr - nC) / hRp                                          # sin(phi - alpha)
    ok_v = np.abs(v) <= 1.0
    asv = np.arcsin(np.clip(v, -1.0, 1.0))
    tanh = np.tan(np.deg2rad(G.SECTOR_HALF_ANGLE_DEG))

    out = {k: [] for k in ("pid", "sector", "row", "y", "z", "s", "T", "Q", "leg", "l")}
    rows = np.broadcast_to(np.arange(G.N_ROWS)[None, :], v.shape)
    for branch in (0, 1):
        dphi_loc = asv if branch == 0 else np.pi - asv          # phi - alpha
        phi = alpha[:, None] + dphi_loc
        cosl = np.cos(dphi_loc)
        yloc = yC - hRp * cosl
        th0 = np.mod(h[ip][:, None] * (phi - phi0[ip][:, None]), 2 * np.pi)
        for turn in (0, 1):
            th = th0 + turn * 2 * np.pi
            l = R[ip][:, None] * th
            zz = p["vz"][ip][:, None] + T[ip][:, None] * l
            ok = ok_v & (l > 0) & (l <= l_max[ip][:, None])
            ok &= np.abs(yloc) <= xr * tanh
            ok &= np.abs(zz) <= G.Z_MAX
            sel = np.nonzero(ok)
            pi = ip[sel[0]]
            sec = ia[sel[0]] + np.where(zz[sel] >= 0.0, 0, 18)
            outward = cosl[sel] > 0
            sgn = np.where(outward, 1.0, -1.0)
            out["pid"].append(pi)
            out["sector"].append(sec)
            out["row"].append(rows[sel])
            out["y"].append(yloc[sel])
            out["z"].append(zz[sel])
            # a returning leg followed towards larger x has direction phi + pi
            out["s"].append(v[sel] * sgn)
            out["T"].append(T[pi] * sgn)
            out["Q"].append(Q[pi] * sgn)
            out["leg"].append(2 * turn + np.where(outward, 0, 1))
            out["l"].append(l[sel])
    return {k: np.concatenate(vv) for k, vv in out.items()}


def _sigma(sig0, sig1, z):
    return sig0 + sig1 * np.abs(z) / G.Z_MAX


def build_event(name, seed, particles, sigma, noise_frac, efficiency, rng,
                sectors=None, smear=True) -> Event:
    x_rows = G.row_x()
    c = _crossings(particles, sectors, x_rows)
    if sectors is not None:
        keep = np.isin(c["sector"], np.asarray(sectors))
        c = {k: v[keep] for k, v in c.items()}
    if efficiency < 1.0:
        keep = rng.uniform(size=len(c["y"])) < efficiency
        c = {k: v[keep] for k, v in c.items()}
    nsig = len(c["y"])
    sy = _sigma(sigma[0], sigma[1], c["z"])
    sz = _sigma(sigma[2], sigma[3], c["z"])
    ym = c["y"] + rng.normal(size=nsig) * sy * (1.0 if smear else 0.0)
    zm = c["z"] + rng.normal(size=nsig) * sz * (1.0 if smear else 0.0)

    nnoise = int(round(noise_frac * nsig))
    sec_pool = np.arange(G.N_SECTORS) if sectors is None else np.asarray(sectors)
    nsec = sec_pool[rng.integers(0, len(sec_pool), nnoise)]
    nrow = rng.integers(0, G.N_ROWS, nnoise)
    ymax = x_rows[nrow].astype(np.float64) * np.tan(np.deg2rad(G.SECTOR_HALF_ANGLE_DEG))
    ny = rng.uniform(-1.0, 1.0, nnoise) * ymax
    nz = rng.uniform(0.0, G.Z_MAX, nnoise) * np.where(nsec < 18, 1.0, -1.0)

    N = nsig + nnoise
    sector = np.concatenate([c["sector"], nsec]).astype(np.uint8)
    row = np.concatenate([c["row"], nrow]).astype(np.uint8)
    y = np.concatenate([ym, ny]).astype(np.float32)
    z = np.concatenate([zm, nz]).astype(np.float32)
    pid = np.concatenate([c["pid"], np.full(nnoise, -1)]).astype(np.int32)
    leg = np.concatenate([c["leg"], np.full(nnoise, -1)]).astype(np.int32)
    truth = np.full((N, 5), np.nan)
    truth[:nsig] = np.stack([c["y"], c["z"], c["s"], c["T"], c["Q"]], axis=1)
    q = (30.0 + rng.exponential(40.0, N)).astype(np.float32)

    perm = rng.permutation(N)
    return Event(name=name, seed=seed, sector=sector[perm], row=row[perm],
                 y=y[perm], z=z[perm], q=q[perm], pid=pid[perm], leg=leg[perm],
                 truth=truth[perm], sigma=tuple(float(s) for s in sigma),
                 particles=particles)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def seed_for(cfg: int, event: int = 0) -> int:
    return SEED_BASE + cfg + 1000 * event


def one_sector_event(seed=None, n_tracks=200) -> Event:
    """One TPC sector (sector 0), 200 origin tracks, pT log-uniform 0.2-5,
    phi uniform over the sector's 20 degrees, 0 <= eta < 0.9 (so that every
    track reaches this A-side sector), sigma_y 0.1 / sigma_z 0.15 cm, full
    efficiency, 5% noise."""
    seed = seed_for(CFG_ONE_SECTOR) if seed is None else seed
    rng = np.random.default_rng(seed)
    pt = _pt_loguniform(rng, n_tracks, 0.2, 5.0)
    p = _particles(rng, n_tracks, pt, 0.0, np.deg2rad(20.0), 0.0, 0.9, kind=0)
    return build_event("one_sector_200", seed, p, G.SIGMA_PP, 0.05, 1.0, rng,
                       sectors=[0])


def pp_event(seed=None, n_primaries=60) -> Event:
    """Full TPC, pp-like: 60 primaries, pT = 0.1 + Exp(0.5 GeV/c), |eta| < 0.9,
    98% per-row efficiency, 5% noise."""
    seed = seed_for(CFG_PP) if seed is None else seed
    rng = np.random.default_rng(seed)
    pt = _pt_exp(rng, n_primaries)
    p = _particles(rng, n_primaries, pt, 0.0, 2 * np.pi, -0.9, 0.9, kind=0)
    return build_event("pp_60", seed, p, G.SIGMA_PP, 0.05, 0.98, rng)


def pbpb_event(seed=None, n_primaries=15000, name=None) -> Event:
    """Full TPC, Pb-Pb shape: n primaries (exp(-pT/0.5) above 0.1 with a
    power-law tail to 20 GeV/c), 20% secondaries from vertices at radius
    0-60 cm, 5% loopers at pT 0.05-0.15, sigma 0.1-0.2 cm, 98% efficiency,
    10% noise."""
    seed = seed_for(CFG_CENTRAL) if seed is None else seed
    rng = np.random.default_rng(seed)
    n_sec = int(round(0.20 * n_primaries))
    n_loop = int(round(0.05 * n_primaries))
    prim = _particles(rng, n_primaries, _pt_exp_tail(rng, n_primaries),
                      0.0, 2 * np.pi, -0.9, 0.9, kind=0)
    sec = _particles(rng, n_sec, _pt_exp_tail(rng, n_sec), 0.0, 2 * np.pi,
                     -0.9, 0.9, kind=1, vertex_radius=60.0)
    loop = _particles(rng, n_loop, rng.uniform(0.05, 0.15, n_loop), 0.0,
                      2 * np.pi, -0.9, 0.9, kind=2)
    p = _concat([prim, sec, loop])
    name = name or f"pbpb_{n_primaries}"
    return build_event(name, seed, p, G.SIGMA_PBPB, 0.10, 0.98, rng)


def central_event(seed=None) -> Event:
    return pbpb_event(seed_for(CFG_CENTRAL) if seed is None else seed, 15000,
                      name="central_pbpb_15000")


def tiny_event(seed, n_tracks=3, pt_lo=0.5, pt_hi=5.0, smear=True, noise_frac=0.0,
               sigma=G.SIGMA_PP) -> Event:
    """A few origin tracks in sector 0, spread evenly in phi and eta so that
    they stay well apart (for brute-force checks of the whole tracker)."""
    rng = np.random.default_rng(seed)
    pt = _pt_loguniform(rng, n_tracks, pt_lo, pt_hi)
    p = _particles(rng, n_tracks, pt, 0.0, 1.0, 0.0, 1.0, kind=0)
    k = np.arange(n_tracks)
    p["phi"] = np.deg2rad(4.0 + 12.0 * (k + 0.5) / n_tracks + rng.uniform(-0.3, 0.3, n_tracks))
    p["eta"] = 0.1 + 0.7 * ((k * 7919) % n_tracks + 0.5) / n_tracks
    return build_event(f"tiny_{n_tracks}", seed, p, sigma, noise_frac, 1.0, rng,
                       sectors=[0], smear=smear)


def membrane_event(seed=20261205, n_tracks=12, noise_frac=0.05) -> Event:
    """Stiff tracks that cross the central membrane inside the TPC: vertex
    z 5-15 cm on the A side, a small negative dip chosen so that z = 0 is
    reached at a transverse radius of 120-200 cm; one track per azimuthal
    sector (12 of the 18), near its centre.  Each leaves a segment in sector
    k (A side) and its continuation in sector k + 18 (C side)."""
    rng = np.random.default_rng(seed)
    pt = rng.uniform(2.0, 5.0, n_tracks)
    p = _particles(rng, n_tracks, pt, 0.0, 1.0, 0.0, 0.1, kind=0)
    k = np.arange(n_tracks)
    p["phi"] = np.deg2rad(20.0 * k + 10.0 + rng.uniform(-3.0, 3.0, n_tracks))
    vz = rng.uniform(5.0, 15.0, n_tracks)
    p["vz"] = vz
    p["eta"] = -np.arcsinh(vz / rng.uniform(120.0, 200.0, n_tracks))
    return build_event("membrane", seed, p, G.SIGMA_PP, noise_frac, 1.0, rng)


def boundary_jet_event(seed=20261206, n_tracks=150) -> Event:
    """Negative tracks of one momentum (pT 0.8 GeV/c, eta 0.3) from vertices
    spread along the beam (z 60 cm either side), launched at 11.4-12.4
    degrees so that they turn across the boundary of sectors 0 and 1 near
    150 cm: every segment pair there passes the merger's cuts on T and Q
    (a segment has up to ~70 such candidates), and only the position match
    picks the partner."""
    rng = np.random.default_rng(seed)
    p = _particles(rng, n_tracks, np.full(n_tracks, 0.8), 0.0, 1.0, 0.0, 1.0, kind=0)
    k = np.arange(n_tracks)
    p["phi"] = np.deg2rad(11.4 + 1.0 * ((k * 37) % n_tracks + 0.5) / n_tracks)
    p["eta"] = np.full(n_tracks, 0.3)
    p["vz"] = -60.0 + 120.0 * (k + 0.5) / n_tracks
    p["charge"] = np.full(n_tracks, -1.0)
    return build_event("boundary_jet", seed, p, G.SIGMA_PP, 0.02, 1.0, rng)


def batch_multiplicities(n_events=64, seed=None) -> np.ndarray:
    seed = seed_for(CFG_BATCH) if seed is None else seed
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(50), np.log(15000), n_events)).astype(np.int64)


def batch_event(e: int, mult: int) -> Event:
    return pbpb_event(seed_for(CFG_BATCH, e), int(mult), name=f"batch_{e}_{mult}")


def serve_event(e: int) -> Event:
    """Event e of the serving mix: 70% pp-like, 25% peripheral (2000
    primaries, Pb-Pb shape), 5% central."""
    seed = seed_for(CFG_SERVE, e)
    u = np.random.default_rng(seed).uniform()
    if u < 0.70:
        return pp_event(seed)
    if u < 0.95:
        return pbpb_event(seed, 2000, name="peripheral_2000")
    return pbpb_event(seed, 15000, name="central_pbpb_15000")


def drift_z(sector, z, eps: float) -> np.ndarray:
    """Cluster z as reconstructed with a drift velocity off by the relative
    eps.  z comes from the drift time to the readout plane at +-z_max of
    each side (sectors 0-17: A side, z > 0; 18-35: C side), so the measured
    z is z (1 + eps) - side eps z_max."""
    side = np.where(np.asarray(sector) < 18, 1.0, -1.0)
    zz = np.asarray(z, np.float64)
    return (zz * (1.0 + eps) - side * eps * G.Z_MAX).astype(np.float32)


def distort_drift(ev: Event, eps: float) -> Event:
    """The event with drift_z applied; truth is unchanged."""
    import dataclasses
    return dataclasses.replace(ev, z=drift_z(ev.sector, ev.z, eps), name=f"{ev.name}_drift{eps:g}")


# ----------------------------------------------------------------------------
# multiple scattering (a model variant: the gas as a uniform scatterer)
# ----------------------------------------------------------------------------

X0_GAS_CM = 31000.0          # radiation length of the drift gas (reading: Ne-based mix)
PION_MASS = 0.13957          # GeV, mass assumed for the scattering law


def ms_theta2_per_cm(x0_cm: float) -> float:
    """k^2 / X0 of the scattering law theta0^2 = k^2 (L / X0) / (beta p)^2
    with k = 13.6 MeV (1 + 0.038 ln(L_ref / X0)) taken at L_ref = 1 cm: the
    plane-angle variance per cm of path is ms_theta2_per_cm / (beta p)^2."""
    k = 0.0136 * (1.0 + 0.038 * np.log(1.0 / x0_cm))
    return k * k / x0_cm


def ms_sector_event(seed, n_tracks=200, x0_cm=X0_GAS_CM, pt_lo=0.2, pt_hi=2.0,
                    noise_frac=0.05, sigma=G.SIGMA_PP) -> Event:
    """One TPC sector (sector 0) with multiple scattering in the gas: tracks
    from the origin (pT log-uniform, phi inside the sector, 0 <= eta < 0.9)
    are followed from pad row to pad row on the exact circle, and at the end
    of each step the direction receives two independent Gaussian kicks of
    variance theta0^2 (bending plane / dip), theta0^2 = k^2/X0 * L / (beta p)^2
    for the path L of that step; |p| is kept (no energy loss), so
    q/pT = q / (p cos(lambda)) follows the dip.  The kick of a step is given
    at its end, so the truth (y, z, sin phi, tan lambda, q/pT) at a crossing
    includes the scattering of the step into it."""
    rng = np.random.default_rng(seed)
    pt = _pt_loguniform(rng, n_tracks, pt_lo, pt_hi)
    q = np.where(rng.uniform(size=n_tracks) < 0.5, -1.0, 1.0)
    phi = rng.uniform(-np.deg2rad(8.0), np.deg2rad(8.0), n_tracks)   # local azimuth
    lam = np.arctan(np.sinh(rng.uniform(0.0, 0.9, n_tracks)))
    p = pt / np.cos(lam)
    b = -G.C_LIGHT * G.BZ_TESLA
    kk = ms_theta2_per_cm(x0_cm)
    X = G.row_x().astype(np.float64)
    tanh = np.tan(np.deg2rad(G.SECTOR_HALF_ANGLE_DEG))
    x = np.zeros(n_tracks)
    y = np.zeros(n_tracks)
    z = np.zeros(n_tracks)
    alive = np.ones(n_tracks, bool)
    rec = {k: [] for k in ("pid", "row", "y", "z", "s", "T", "Q")}
    pid_all = np.arange(n_tracks)
    for r in range(G.N_ROWS):
        Q = q / (p * np.cos(lam))          # q / pT, pT = p cos(lambda)
        s0 = np.sin(phi)
        dx = X[r] - x
        s1 = s0 + b * Q * dx
        alive &= np.abs(s1) < 0.999
        s1 = np.clip(s1, -0.999, 0.999)
        c0, c1 = np.sqrt(1 - s0 * s0), np.sqrt(1 - s1 * s1)
        y = y + dx * (s0 + s1) / (c0 + c1)
        dphi = np.arcsin(s1) - np.arcsin(s0)
        bq = b * Q
        with np.errstate(divide="ignore", invalid="ignore"):
            lperp = np.where(np.abs(bq) > 1e-12, dphi / bq, dx * np.sqrt(1 + ((s0 + s1) / (c0 + c1)) ** 2))
        T = np.tan(lam)
        z = z + T * lperp
        x = np.full(n_tracks, X[r])
        phi = np.arcsin(s1)
        # the step's scattering, at its end (before this row's crossing is
        # recorded, as the fit adds a step's noise before that row's update)
        L = lperp * np.sqrt(1 + T * T)
        beta2p2 = p * p * p * p / (p * p + PION_MASS ** 2)        # (beta p)^2
        th = np.sqrt(kk * np.abs(L) / beta2p2)
        phi = phi + th * rng.normal(size=n_tracks) / np.cos(lam)
        lam = lam + th * rng.normal(size=n_tracks)
        alive &= (np.abs(y) <= X[r] * tanh) & (np.abs(z) <= G.Z_MAX) & (np.abs(np.sin(phi)) < 0.999)
        sel = np.nonzero(alive)[0]
        for k, v in (("pid", pid_all), ("row", np.full(n_tracks, r)), ("y", y), ("z", z),
                     ("s", np.sin(phi)), ("T", np.tan(lam)), ("Q", q / (p * np.cos(lam)))):
            rec[k].append(v[sel])
    c = {k: np.concatenate(v) for k, v in rec.items()}
    nsig = len(c["y"])
    keep = np.ones(nsig, bool)
    sy = _sigma(sigma[0], sigma[1], c["z"])
    sz = _sigma(sigma[2], sigma[3], c["z"])
    ym = c["y"] + rng.normal(size=nsig) * sy
    zm = c["z"] + rng.normal(size=nsig) * sz
    nnoise = int(round(noise_frac * nsig))
    nrow = rng.integers(0, G.N_ROWS, nnoise)
    ny = rng.uniform(-1.0, 1.0, nnoise) * X[nrow] * tanh
    nz = rng.uniform(0.0, G.Z_MAX, nnoise)
    N = nsig + nnoise
    sector = np.zeros(N, np.uint8)
    row = np.concatenate([c["row"], nrow]).astype(np.uint8)
    yy = np.concatenate([ym, ny]).astype(np.float32)
    zz = np.concatenate([zm, nz]).astype(np.float32)
    pid = np.concatenate([c["pid"], np.full(nnoise, -1)]).astype(np.int32)
    leg = np.concatenate([np.zeros(nsig, np.int32), np.full(nnoise, -1)]).astype(np.int32)
    truth = np.full((N, 5), np.nan)
    truth[:nsig] = np.stack([c["y"], c["z"], c["s"], c["T"], c["Q"]], axis=1)
    qq = (30.0 + rng.exponential(40.0, N)).astype(np.float32)
    perm = rng.permutation(N)
    del keep
    particles = dict(vx=np.zeros(n_tracks), vy=np.zeros(n_tracks), vz=np.zeros(n_tracks), pt=pt,
                     phi=phi, eta=np.arcsinh(np.tan(lam)), charge=q,
                     kind=np.zeros(n_tracks, np.int8))
    return Event(name=f"ms_sector_{n_tracks}", seed=seed, sector=sector[perm], row=row[perm],
                 y=yy[perm], z=zz[perm], q=qq[perm], pid=pid[perm], leg=leg[perm],
                 truth=truth[perm], sigma=tuple(float(s) for s in sigma), particles=particles)
