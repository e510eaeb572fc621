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


def lens_analytic(theta1: float, theta2: float, area: float):
    """Lens length and cap heights of Eq. (23) for contact angles theta1, theta2 (radians)
    and lens area `area`: D = 2 sqrt(A / sum_i (theta_i / sin theta_i - cos theta_i) /
    sin theta_i), h_i = (D/2) (1 - cos theta_i) / sin theta_i."""
    s = sum((t / math.sin(t) - math.cos(t)) / math.sin(t) for t in (theta1, theta2))
    D = 2.0 * math.sqrt(area / s)
    return D, 0.5 * D * (1 - math.cos(theta1)) / math.sin(theta1), 0.5 * D * (1 - math.cos(theta2)) / math.sin(theta2)


def _crossing(v: np.ndarray, level: float, i0: int, step: int) -> float:
    """Fractional index where the 1-d profile v first crosses `level` walking from i0 in
    direction step (+1 or -1), by linear interpolation between the two bracketing nodes."""
    i = i0
    while 0 <= i + step < len(v):
        a, b = v[i] - level, v[i + step] - level
        if a == 0:
            return float(i)
        if a * b < 0:
            return i + step * a / (a - b)
        i += step
    raise ValueError("no crossing")


def lens_geometry(rho: np.ndarray, y_guess: float, x_far: int = 0):
    """Length D and cap heights of a lens of fluid 0 on the flat interface between fluid 1
    (below) and fluid 2 (above), measured on the concentration fields: the flat interface
    height y_i where c_1 = c_2 in column x_far (away from the lens); D between the two
    points where c_0 = 1/2 along the line y = y_i; the heights where c_0 = 1/2 above and
    below y_i along the lens's middle column.  Returns (D, h_up, h_down, y_i)."""
    c = rho / rho.sum(0)
    ny, nx = c.shape[1:]
    y_i = _crossing(c[1, :, x_far] - c[2, :, x_far], 0.0, int(y_guess) - 10, +1)
    j = int(math.floor(y_i))
    t = y_i - j
    row = (1 - t) * c[0, j] + t * c[0, j + 1]
    xm = int(np.argmax(row))
    xl = _crossing(row, 0.5, xm, -1)
    xr = _crossing(row, 0.5, xm, +1)
    xc = 0.5 * (xl + xr)
    i = int(math.floor(xc))
    s = xc - i
    col = (1 - s) * c[0, :, i] + s * c[0, :, i + 1]
    y_top = _crossing(col, 0.5, j + 1, +1) if col[j + 1] > 0.5 else y_i
    y_bot = _crossing(col, 0.5, j, -1) if col[j] > 0.5 else y_i
    return xr - xl, y_top - y_i, y_i - y_bot, y_i


def gjd_geometry(Rr: float, Rg: float, Rb: float, drg: float, sigma_rg: float = 0.01) -> dict:
    """General Janus droplet of Sec. 4 (fluids r, g inside b): from the radii of the rb, gb
    and rg interfaces and the distance d_rg between the rb and gb centres, the half central
    angles and d_gb (Eqs. gjd_01-03), the Neumann angles phi_kl (Eqs. gjd_04/05, chosen by
    where the gb centre lies) and, with sigma_rg, the other two tensions by the law of sines
    (Eq. gjd_06)."""
    tg = math.acos((Rg * Rg + drg * drg - Rr * Rr) / (2 * Rg * drg))
    chord = Rg * math.sin(tg)
    tb = math.asin(chord / Rb)
    tr = math.asin(chord / Rr)
    dgb = Rg * math.cos(tg) + Rb * math.cos(tb)
    if Rg * math.cos(tg) >= drg:
        prb, pgb = math.pi / 2 - tr + tg, math.pi - tr - tb
    else:
        prb, pgb = tb + tg, tr - tb
    prg = math.pi - prb - pgb
    k = sigma_rg / math.sin(prg)
    return {"theta_g": tg, "theta_r": tr, "theta_b": tb, "d_gb": dgb, "phi_rb": prb, "phi_gb": pgb,
            "phi_rg": prg, "sigma_gb": k * math.sin(pgb), "sigma_rb": k * math.sin(prb)}


def interface_points(c: np.ndarray, k: int, l: int, third_max: float = 0.05) -> np.ndarray:
    """Points of the k-l interface: where c_k - c_l changes sign between horizontally or
    vertically adjacent nodes (linear interpolation), at node pairs where the third fluid's
    concentration stays below third_max.  Returns an (n, 2) array of (x, y)."""
    m = 3 - k - l
    d = c[k] - c[l]
    pts = []
    for axis in (0, 1):
        a, b = (d[:-1, :], d[1:, :]) if axis == 0 else (d[:, :-1], d[:, 1:])
        ma = c[m][:-1, :] if axis == 0 else c[m][:, :-1]
        mb = c[m][1:, :] if axis == 0 else c[m][:, 1:]
        sel = (a * b < 0) & (ma < third_max) & (mb < third_max)
        jj, ii = np.nonzero(sel)
        t = a[sel] / (a[sel] - b[sel])
        if axis == 0:
            pts.append(np.stack([ii.astype(float), jj + t], 1))
        else:
            pts.append(np.stack([ii + t, jj.astype(float)], 1))
    return np.concatenate(pts)


def fit_circle(p: np.ndarray):
    """Least-squares circle through the points p (algebraic fit of x^2 + y^2 + a x + b y + e
    = 0).  Returns (xc, yc, R)."""
    A = np.column_stack([p[:, 0], p[:, 1], np.ones(len(p))])
    rhs = -(p[:, 0] ** 2 + p[:, 1] ** 2)
    (a, b, e), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    xc, yc = -a / 2, -b / 2
    return xc, yc, math.sqrt(xc * xc + yc * yc - e)


def contact_length(rho: np.ndarray, y_mid: float, third: int = 2) -> float:
    """Length of the contact between the two other fluids across the line y = y_mid: the
    fraction not of fluid `third`, summed along the two lattice rows next to the line and
    averaged over them (a point contact leaves only the diffuse tails, about 9 nodes at
    R = 60)."""
    c = rho / rho.sum(0)
    rows = [int(math.floor(y_mid)), int(math.ceil(y_mid))]
    return float(np.mean([(1.0 - c[third, r]).sum() for r in rows]))


def mixed_nodes(rho: np.ndarray, k: int, l: int, level: float = 0.2) -> int:
    """Nodes where both fluids k and l hold more than `level` of the mixture: a measure of
    the length of the k-l interface (about its length times its width)."""
    c = rho / rho.sum(0)
    return int((np.minimum(c[k], c[l]) > level).sum())


def circle_intersections(c1, c2):
    """The two intersection points of circles (xc, yc, R) c1 and c2 (empty if they miss)."""
    (x1, y1, r1), (x2, y2, r2) = c1, c2
    d = math.hypot(x2 - x1, y2 - y1)
    if d == 0 or d > r1 + r2 or d < abs(r1 - r2):
        return []
    a = (r1 * r1 - r2 * r2 + d * d) / (2 * d)
    h = math.sqrt(max(r1 * r1 - a * a, 0.0))
    xm, ym = x1 + a * (x2 - x1) / d, y1 + a * (y2 - y1) / d
    return [(xm + h * (y2 - y1) / d, ym - h * (x2 - x1) / d),
            (xm - h * (y2 - y1) / d, ym + h * (x2 - x1) / d)]


def _bilinear(f: np.ndarray, x: float, y: float) -> float:
    i, j = int(math.floor(x)), int(math.floor(y))
    s, t = x - i, y - j
    return float((1 - s) * (1 - t) * f[j, i] + s * (1 - t) * f[j, i + 1]
                 + (1 - s) * t * f[j + 1, i] + s * t * f[j + 1, i + 1])


def junction_phase_angles(rho: np.ndarray, near: tuple = (6.0, 30.0), probe: float = 8.0):
    """Phase angles at the two triple junctions of a droplet of fluids 0 and 1 in fluid 2
    (a Janus droplet).  Circles are fitted to the three interfaces (points where two
    concentrations cross, away from the third fluid); the junctions are the intersections of
    the 0-1 and 0-2 circles (the 0-2 and 1-2 circles coincide for a perfect Janus droplet,
    the 0-1 circle meets them at right angles there).  At each junction every interface
    leaves along its circle's
    tangent, pointed toward that interface's points at distances `near` from the junction;
    the three tangents split the full turn into three angles, each assigned to the fluid
    found `probe` nodes out along its bisector.  Returns [{fluid: angle in radians}, ...]."""
    c = rho / rho.sum(0)
    pairs = {"rb": (0, 2), "gb": (1, 2), "rg": (0, 1)}
    pts = {n: interface_points(c, k, l) for n, (k, l) in pairs.items()}
    fits = {n: fit_circle(p) for n, p in pts.items()}
    out = []
    for J in circle_intersections(fits["rg"], fits["rb"]):
        dirs = []
        for n in pairs:
            xc, yc, _ = fits[n]
            rx, ry = J[0] - xc, J[1] - yc
            t = np.array([-ry, rx]) / math.hypot(rx, ry)
            dist = np.hypot(pts[n][:, 0] - J[0], pts[n][:, 1] - J[1])
            sel = pts[n][(dist > near[0]) & (dist < near[1])]
            if len(sel) == 0:
                raise ValueError(f"no {n} interface points near the junction {J}")
            if np.dot(sel.mean(0) - np.array(J), t) < 0:
                t = -t
            dirs.append(math.atan2(t[1], t[0]))
        dirs.sort()
        angles = {}
        for q in range(3):
            a0, a1 = dirs[q], dirs[(q + 1) % 3] + (2 * math.pi if q == 2 else 0.0)
            mid = 0.5 * (a0 + a1)
            x, y = J[0] + probe * math.cos(mid), J[1] + probe * math.sin(mid)
            fluid = int(np.argmax([_bilinear(c[k], x, y) for k in range(3)]))
            angles[fluid] = a1 - a0
        out.append(angles)
    return out


def pjd_geometry(area_fraction: float, R: float) -> dict:
    """Perfect Janus droplet (Sec. 4, Eq. pjd): the red and green fluids fill a disk of
    radius R = R_r = R_g, split by the rg interface, an arc of radius R_b centred d_gb above
    the disk's centre.  theta_g solves
      A_r / (A_r + A_g) = [theta - sin cos + tan^2 theta (pi/2 - theta - sin cos)] / pi
    (bisection on (0, pi/2), where the right side rises from 0 to 1/2), R_b = R tan theta_g and
    d_gb = R cos theta_g + R_b cos theta_b with R sin theta_g = R_b sin theta_b."""
    def frac(t):
        sc = math.sin(t) * math.cos(t)
        return (t - sc + math.tan(t) ** 2 * (math.pi / 2 - t - sc)) / math.pi
    lo, hi = 1e-9, math.pi / 2 - 1e-12
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if frac(mid) < area_fraction:
            lo = mid
        else:
            hi = mid
    tg = 0.5 * (lo + hi)
    Rb = R * math.tan(tg)
    tb = math.asin(min(1.0, R * math.sin(tg) / Rb))
    return {"theta_g": tg, "theta_b": tb, "R_b": Rb, "d_gb": R * math.cos(tg) + Rb * math.cos(tb)}


def kissing_chord(R: float, sigma_rg: float, sigma_gb: float) -> float:
    """Length L_rg of the flat interface between two equal droplets of radius R (fluids 0 and
    1, sigma_rb = sigma_gb) at equilibrium: their centres sit d_rg = R sigma_rg / sigma_gb apart
    (Sec. 4, Eq. drg) while sigma_gb > sigma_rg / 2, so the shared chord is
    2 sqrt(R^2 - d_rg^2 / 4); at and below the kissing state it is 0."""
    if sigma_gb <= sigma_rg / 2:
        return 0.0
    d = R * sigma_rg / sigma_gb
    return 2.0 * math.sqrt(R * R - d * d / 4.0)


def engulfed_rb_arc(Rr: float, Rg: float, sigma_rb: float, sigma_gb: float) -> tuple:
    """Near-critical engulfing (Sec. 4): a droplet of fluid 0 (radius Rr) partly engulfed by
    one of fluid 1 (radius Rg), sigma_rg = sigma_gb.  Returns (d_rg, L_rb): the distance of the
    centres, d_rg^2 = Rr^2 + Rg^2 - 2 Rr Rg cos(alpha) with cos(alpha) = sigma_rb / (2 sigma_gb)
    (d_rg = Rg - Rr at and beyond the critical state sigma_rb = 2 sigma_gb), and the length of
    fluid 0's arc outside fluid 1, 2 Rr (pi - phi) with phi the angle at fluid 0's centre
    between its junctions and fluid 1's centre."""
    if sigma_rb >= 2 * sigma_gb:
        return Rg - Rr, 0.0
    ca = sigma_rb / (2 * sigma_gb)
    d = math.sqrt(Rr * Rr + Rg * Rg - 2 * Rr * Rg * ca)
    phi = math.acos((Rr * Rr + d * d - Rg * Rg) / (2 * Rr * d))
    return d, 2 * Rr * (math.pi - phi)


def arc_length(points: np.ndarray) -> float:
    """Length of the circular arc through `points` (an (n, 2) array): the fitted circle's radius
    times the angular extent of the points about its centre (0 for fewer than 3 points)."""
    if len(points) < 3:
        return 0.0
    xc, yc, R = fit_circle(points)
    ang = np.sort(np.arctan2(points[:, 1] - yc, points[:, 0] - xc))
    gaps = np.diff(np.concatenate([ang, ang[:1] + 2 * math.pi]))
    return R * (2 * math.pi - gaps.max())
