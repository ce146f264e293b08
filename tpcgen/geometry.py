"""TPC geometry and detector constants shared by the synthetic-event generator.

This module describes the detector only (where the pad rows are, the field,
the acceptance).  It holds none of the tracker's arithmetic: both the CPU
oracle and the HIP library receive these numbers as *inputs* (a row-radius
table, the field, the acceptance, the cluster-error model).

Readings (the paper names a 36-sector, 159-pad-row TPC read out by detector
links, Section 2, but gives no radii):
  * 63 inner rows at 0.75 cm pitch from 85.225 cm, 64 rows at 1.0 cm from
    135.1 cm and 32 rows at 1.5 cm from 199.35 cm (last row 245.85 cm);
  * sectors 0-17 cover z >= 0 (A side), 18-35 cover z <= 0 (C side), each
    20 degrees wide, sector s centred on azimuth ((s mod 18) + 0.5) * 20 deg;
  * B_z = 0.5 T, drift length 250 cm.
"""
from __future__ import annotations

import numpy as np

N_SECTORS = 36
N_ROWS = 159
SECTOR_HALF_ANGLE_DEG = 10.0
Z_MAX = 250.0
BZ_TESLA = 0.5
R_EXIT = 250.0            # outer field-cage radius: particles leave the drift volume here
C_LIGHT = 0.00299792458   # GeV / (T cm): p_T = C_LIGHT * B * R for unit charge

# cluster-error models (sigma0, sigma1) meaning sigma(z) = sigma0 + sigma1*|z|/Z_MAX
SIGMA_PP = (0.1, 0.0, 0.15, 0.0)        # sigma_y = 0.1 cm, sigma_z = 0.15 cm
SIGMA_PBPB = (0.1, 0.1, 0.1, 0.1)       # 0.1 ... 0.2 cm in both y and z


def row_x() -> np.ndarray:
    """Pad-row radii X_r as float32 (the tracker sees exactly these values)."""
    r = np.arange(N_ROWS, dtype=np.float64)
    x = np.where(r < 63, 85.225 + 0.75 * r,
                 np.where(r < 127, 135.1 + 1.0 * (r - 63), 199.35 + 1.5 * (r - 127)))
    return x.astype(np.float32)


def sector_alpha(sector) -> np.ndarray:
    """Azimuth (radians) of the centre line of a sector."""
    s = np.asarray(sector)
    return np.deg2rad(((s % 18) + 0.5) * 20.0)


def tan_half_angle() -> np.float32:
    return np.float32(np.tan(np.deg2rad(SECTOR_HALF_ANGLE_DEG)))


def geometry_dict(sigma=SIGMA_PP) -> dict:
    """Everything the tracker is told about the detector, as plain numbers."""
    return dict(
        n_sectors=N_SECTORS,
        n_rows=N_ROWS,
        row_x=row_x(),
        bz_tesla=np.float32(BZ_TESLA),
        tan_half_angle=tan_half_angle(),
        z_max=np.float32(Z_MAX),
        sigma_y0=np.float32(sigma[0]), sigma_y1=np.float32(sigma[1]),
        sigma_z0=np.float32(sigma[2]), sigma_z1=np.float32(sigma[3]),
    )
