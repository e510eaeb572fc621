"""Measurements on density fields used by the physics tests (test-side helpers)."""
from __future__ import annotations

import math

import numpy as np


def radius_map(nx: int, ny: int, xc: float, yc: float) -> np.ndarray:
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    return np.sqrt((x - xc) ** 2 + (y - yc) ** 2)


def pressure(rho: np.ndarray) -> np.ndarray:
    """p = c_s^2 rho with c_s^2 = 1/3."""
    return rho.sum(0) / 3.0


def compound_laplace(rho: np.ndarray, xc: float, yc: float, sigma_rg: float, sigma_gb: float):
    """Pressure jumps of a compound droplet (fluid 0 core, fluid 1 shell, fluid 2 outside):
    radii from the conserved colour areas, p_in averaged over r <= R_r/2, the shell over
    |r - (R_r+R_g)/2| <= (R_g-R_r)/4, outside over r >= R_g + 15.  Returns a dict with the
    jumps, radii and the relative error of Eq. (27)."""
    ny, nx = rho.shape[1:]
    c = rho / rho.sum(0)
    Rr = math.sqrt(c[0].sum() / math.pi)
    Rg = math.sqrt((c[0] + c[1]).sum() / math.pi)
    r = radius_map(nx, ny, xc, yc)
    p = pressure(rho)
    p_in = p[r <= Rr / 2].mean()
    p_sh = p[np.abs(r - (Rr + Rg) / 2) <= (Rg - Rr) / 4].mean()
    p_out = p[r >= Rg + 15].mean()
    dp_rg, dp_gb = p_in - p_sh, p_sh - p_out
    eps = abs(dp_gb * Rg + dp_rg * Rr - (sigma_gb + sigma_rg)) / (sigma_gb + sigma_rg)
    return {"Rr": Rr, "Rg": Rg, "dp_rg": dp_rg, "dp_gb": dp_gb, "dp_total": p_in - p_out,
            "eps": eps}
