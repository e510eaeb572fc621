"""Seeded synthetic inputs for the ternary colour-gradient LBM.

This module holds the input recipes only: geometry (disks, shells, half-disks,
flat layers), the interface-noise rule, a counter-based generator and
parameter sets.  It contains none of the method's arithmetic and is the one
module that both the HIP path's tests and the oracle's tests import.

Conventions: density fields are ``rho[3, ny, nx]`` float64 (fluids 0, 1, 2 are
the paper's red, green, blue), node (x, y) sits at integer coordinates,
0-based; a node is inside a disk of centre (xc, yc) and radius R when
(x - xc)^2 + (y - yc)^2 <= R^2, and where shapes overlap the first-listed one
wins.  ``sigma = (sigma_rg, sigma_rb, sigma_gb)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs start..start+n-1 of SplitMix64 (Steele, Lea, Flood 2014) from ``seed``.

    Counter form: state_j = seed + (j + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then the
    published 30/27/31 xor-shift-multiply finaliser."""
    with np.errstate(over="ignore"):
        j = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + j * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, n: int, start: int = 0) -> np.ndarray:
    """u = (x >> 11) * 2^-53 in [0, 1)."""
    return (splitmix64(seed, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclass
class Workload:
    """A synthetic problem: lattice, parameters and initial density (and velocity) fields."""
    name: str
    nx: int
    ny: int
    sigma: tuple
    tau: tuple = (1.0, 1.0, 1.0)
    rho0: tuple = (1.0, 1.0, 1.0)
    beta0: float = 0.7
    steps: int = 0
    rho: np.ndarray | None = None
    u: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


# ------------------------------------------------------------------ geometry
def _grid(nx: int, ny: int):
    y, x = np.mgrid[0:ny, 0:nx]
    return x.astype(np.float64), y.astype(np.float64)


def label_disks(nx: int, ny: int, disks, background: int = 2) -> np.ndarray:
    """Fluid label per node; ``disks`` = [(fluid, xc, yc, R), ...], first listed wins."""
    x, y = _grid(nx, ny)
    lab = np.full((ny, nx), background, dtype=np.int64)
    done = np.zeros((ny, nx), dtype=bool)
    for fluid, xc, yc, R in disks:
        inside = ((x - xc) ** 2 + (y - yc) ** 2 <= R * R) & ~done
        lab[inside] = fluid
        done |= inside
    return lab


def rho_from_labels(lab: np.ndarray) -> np.ndarray:
    rho = np.zeros((3,) + lab.shape)
    for k in range(3):
        rho[k][lab == k] = 1.0
    return rho


def add_interface_noise(rho: np.ndarray, lab: np.ndarray, disks, seed: int,
                        amp: float = 0.01, band: float = 1.5) -> np.ndarray:
    """At nodes within ``band`` of a disk boundary, every fluid absent at the node gets
    ``amp * u`` (u from SplitMix64 draw (k*ny + y)*nx + x) and the node's own fluid gets
    1 minus their sum, so the total stays 1 and every density stays >= 0."""
    ny, nx = lab.shape
    x, y = _grid(nx, ny)
    near = np.zeros((ny, nx), dtype=bool)
    for _, xc, yc, R in disks:
        d = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
        near |= np.abs(d - R) <= band
    u = uniform01(seed, 3 * nx * ny).reshape(3, ny, nx)
    out = rho.copy()
    total_noise = np.zeros((ny, nx))
    for k in range(3):
        m = near & (lab != k)
        out[k][m] = amp * u[k][m]
        total_noise[m] += amp * u[k][m]
    for k in range(3):
        m = near & (lab == k)
        out[k][m] = 1.0 - total_noise[m]
    return out


def tanh_disk(nx: int, ny: int, xc: float, yc: float, R: float, xi: float) -> np.ndarray:
    """0.5 + 0.5 tanh((R - |x - x_c|)/xi): the initial profile of the stability-diagram runs."""
    x, y = _grid(nx, ny)
    return 0.5 + 0.5 * np.tanh((R - np.sqrt((x - xc) ** 2 + (y - yc) ** 2)) / xi)


# ------------------------------------------------------------------ workloads
def two_droplets_64() -> Workload:
    """64x64 periodic, fluid 0 and fluid 1 disks of radius 12 centred at (20,32) and (44,32)
    in fluid 2, all densities 1, tau = 1, sigma = 0.01, zero velocity, 2000 steps.
    (The centres are 2R apart, so the disks touch at (32,32); fluid 0 wins there.)"""
    disks = [(0, 20.0, 32.0, 12.0), (1, 44.0, 32.0, 12.0)]
    rho = rho_from_labels(label_disks(64, 64, disks))
    return Workload("two_droplets_64", 64, 64, (0.01, 0.01, 0.01), steps=2000, rho=rho,
                    meta={"disks": disks})


def separated_droplets_64() -> Workload:
    disks = [(0, 16.0, 32.0, 12.0), (1, 48.0, 32.0, 12.0)]
    rho = rho_from_labels(label_disks(64, 64, disks))
    return Workload("separated_droplets_64", 64, 64, (0.01, 0.01, 0.01), steps=2000, rho=rho,
                    meta={"disks": disks})


def compound_droplet(n: int = 256, r_in: float = 30.0, r_out: float = 60.0,
                     sigma_rg: float = 0.01, sigma_gb: float = 0.01, sigma_rb: float | None = None,
                     tau=(1.0, 1.0, 1.0), steps: int = 20000) -> Workload:
    """Concentric disk of fluid 0 (radius r_in) in a fluid-1 annulus (radius r_out) in fluid 2,
    centred at (n/2, n/2); sigma_rb defaults to sigma_rg + sigma_gb."""
    if sigma_rb is None:
        sigma_rb = sigma_rg + sigma_gb
    c = n / 2.0
    disks = [(0, c, c, r_in), (1, c, c, r_out)]
    rho = rho_from_labels(label_disks(n, n, disks))
    return Workload(f"compound_{n}", n, n, (sigma_rg, sigma_rb, sigma_gb), tuple(tau), steps=steps,
                    rho=rho, meta={"disks": disks, "r_in": r_in, "r_out": r_out, "centre": c})


def single_droplet(n: int, R: float, sigma: float = 0.01, tau=(1.0, 1.0, 1.0),
                   fluid: int = 0) -> Workload:
    c = n / 2.0
    disks = [(fluid, c, c, R)]
    rho = rho_from_labels(label_disks(n, n, disks))
    return Workload(f"droplet_{n}_R{R}", n, n, (sigma, sigma, sigma), tuple(tau), rho=rho,
                    meta={"disks": disks, "R": R, "centre": c})


def double_droplet(n: int, R: float, ratio_rg: float, ratio_rb: float, sigma_gb: float = 0.01,
                   seed: int = 1808, noise: bool = True, tau=(1.0, 1.0, 1.0),
                   steps: int = 50000) -> Workload:
    """Two tangent disks of radius R (fluid 0 above, fluid 1 below the centre line) in fluid 2,
    sigma_rg = ratio_rg * sigma_gb, sigma_rb = ratio_rb * sigma_gb, optional interface noise."""
    c = n / 2.0 - 0.5
    disks = [(0, c, c + R, R), (1, c, c - R, R)]
    lab = label_disks(n, n, disks)
    rho = rho_from_labels(lab)
    if noise:
        rho = add_interface_noise(rho, lab, disks, seed)
    return Workload(f"double_droplet_{n}", n, n,
                    (ratio_rg * sigma_gb, ratio_rb * sigma_gb, sigma_gb), tuple(tau), steps=steps,
                    rho=rho, meta={"disks": disks, "R": R})


def janus_halves(n: int = 256, R: float = 40.0, sigma=(0.006, 0.010, 0.012), tau=(0.8, 0.8, 0.8),
                 steps: int = 5000) -> Workload:
    """Disk of radius R at the centre; fluid 0 on the half x < centre, fluid 1 on x >= centre."""
    c = n / 2.0
    x, y = _grid(n, n)
    inside = (x - c) ** 2 + (y - c) ** 2 <= R * R
    lab = np.full((n, n), 2, dtype=np.int64)
    lab[inside & (x < c)] = 0
    lab[inside & (x >= c)] = 1
    rho = rho_from_labels(lab)
    return Workload(f"janus_{n}", n, n, tuple(sigma), tuple(tau), steps=steps, rho=rho,
                    meta={"R": R, "centre": c})


def loss_target(rho1: np.ndarray, seed: int = 5550, amp: float = 0.05) -> np.ndarray:
    """Seeded target field rho* = rho1 + amp * eta, eta ~ U(-1, 1) from SplitMix64(seed)."""
    eta = 2.0 * uniform01(seed, rho1.size).reshape(rho1.shape) - 1.0
    return rho1 + amp * eta


BATCH_SIDES = (128, 192, 256, 384, 512)


def morphology_batch(count: int = 64, seed: int = 855, sigma_gb: float = 0.01):
    """Instance j: (sigma_rg/sigma_gb, sigma_rb/sigma_gb) = (0.25(1 + j mod 8), 0.25(1 + j div 8)),
    side from {128,...,512} by SplitMix64(seed) draw j mod 5, two tangent disks of radius side/6
    at (c -+ side/6, c), tau = 1."""
    draws = splitmix64(seed, count)
    out = []
    for j in range(count):
        side = BATCH_SIDES[int(draws[j] % np.uint64(5))]
        r12 = 0.25 * (1 + j % 8)
        r13 = 0.25 * (1 + j // 8)
        R = side / 6.0
        c = side / 2.0
        disks = [(0, c - R, c, R), (1, c + R, c, R)]
        rho = rho_from_labels(label_disks(side, side, disks))
        out.append(Workload(f"morph_{j}", side, side, (r12 * sigma_gb, r13 * sigma_gb, sigma_gb),
                            (1.0, 1.0, 1.0), steps=10000, rho=rho,
                            meta={"disks": disks, "r12": r12, "r13": r13}))
    return out


def droplet_tiling(n: int = 4096, cell: int = 256, R: float = 40.0, seed: int = 1808,
                   sigma=(0.01, 0.01, 0.01), tau=(1.0, 1.0, 1.0)) -> Workload:
    """n x n periodic lattice tiled by cells of cell x cell nodes; each cell holds two tangent
    disks of radius R (fluid 0 centred at (c - R, c), fluid 1 at (c + R, c), c the cell centre)
    in fluid 2, with interface noise.  Built per cell, so memory stays small."""
    base_disks = [(0, cell / 2.0 - R, cell / 2.0, R), (1, cell / 2.0 + R, cell / 2.0, R)]
    lab_cell = label_disks(cell, cell, base_disks)
    rho_cell = rho_from_labels(lab_cell)
    reps = n // cell
    rho = np.tile(rho_cell, (1, reps, reps))
    lab = np.tile(lab_cell, (reps, reps))
    # noise over the whole lattice with one counter stream
    x, y = _grid(cell, cell)
    near_cell = np.zeros((cell, cell), dtype=bool)
    for _, xc, yc, r in base_disks:
        near_cell |= np.abs(np.sqrt((x - xc) ** 2 + (y - yc) ** 2) - r) <= 1.5
    near = np.tile(near_cell, (reps, reps))
    iy, ix = np.nonzero(near)
    tot = np.zeros(iy.shape)
    for k in range(3):
        # same draw numbering as add_interface_noise: (k*ny + y)*nx + x
        idx = (k * n + iy).astype(np.uint64) * np.uint64(n) + ix.astype(np.uint64)
        u = _uniform_at(seed, idx)
        absent = lab[iy, ix] != k
        v = np.where(absent, 0.01 * u, 0.0)
        rho[k, iy, ix] = np.where(absent, v, rho[k, iy, ix])
        tot += v
    for k in range(3):
        own = lab[iy, ix] == k
        rho[k, iy, ix] = np.where(own, 1.0 - tot, rho[k, iy, ix])
    return Workload(f"droplet_tiling_{n}", n, n, tuple(sigma), tuple(tau), rho=rho,
                    meta={"cell": cell, "R": R, "seed": seed})


def _uniform_at(seed: int, idx: np.ndarray) -> np.ndarray:
    """SplitMix64 output number idx (0-based) for arbitrary indices, mapped to [0, 1)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def random_mixture(nx: int, ny: int, seed: int, tiny_fraction: float = 0.15) -> np.ndarray:
    """Random positive densities in [0.05, 1.05) per fluid; a fraction of (node, fluid) entries
    is replaced by tiny values (1e-9..1e-6) or exact zeros so that every branch of the
    concentration factor and of the colour-gradient guard is visited."""
    u = uniform01(seed, 3 * nx * ny).reshape(3, ny, nx)
    v = uniform01(seed + 1, 3 * nx * ny).reshape(3, ny, nx)
    rho = 0.05 + u
    tiny = v < tiny_fraction
    rho = np.where(tiny, np.where(v < tiny_fraction / 3, 0.0, 1e-9 + 1e-6 * u), rho)
    # at least one fluid present at every node
    rho[0] = np.where(rho.sum(axis=0) <= 0.0, 0.5, rho[0])
    return rho


def random_mixture_3d(nx: int, ny: int, nz: int, seed: int, tiny_fraction: float = 0.15) -> np.ndarray:
    """random_mixture on an nx x ny x nz lattice: rho [3, nz, ny, nx]."""
    return random_mixture(nx, ny * nz, seed, tiny_fraction).reshape(3, nz, ny, nx)


def spheres(nx: int, ny: int, nz: int, balls) -> np.ndarray:
    """Densities [3, nz, ny, nx] of fluid-2 background with balls (fluid, cx, cy, cz, R); later
    balls win where they overlap."""
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    lab = np.full((nz, ny, nx), 2, dtype=np.int64)
    for k, cx, cy, cz, R in balls:
        lab[(x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= R * R] = k
    return rho_from_labels(lab)


def random_velocity(nx: int, ny: int, seed: int, amp: float = 0.02) -> np.ndarray:
    return amp * (2.0 * uniform01(seed, 2 * nx * ny).reshape(2, ny, nx) - 1.0)


def pie(n: int = 8) -> np.ndarray:
    """Three 120-degree sectors around the lattice centre (a triple junction)."""
    x, y = _grid(n, n)
    ang = np.mod(np.arctan2(y - (n - 1) / 2.0, x - (n - 1) / 2.0), 2 * np.pi)
    lab = np.minimum((ang / (2 * np.pi / 3)).astype(np.int64), 2)
    return rho_from_labels(lab)


def stratified_lens(n: int = 160, R: float = 20.0, sigma_rg: float = 0.01, sigma_rb: float = 0.01,
                    sigma_gb: float = 0.01, tau: float = 0.8, steps: int = 0) -> Workload:
    """A disk of fluid 0 (radius R) at the centre of an n x n periodic lattice whose lower
    half (y < n/2) is fluid 1 and upper half fluid 2: the droplet between two stratified
    fluids that spreads into a lens."""
    c = (n - 1) / 2.0
    lab = label_disks(n, n, [(0, c, c, R)], background=2)
    _, y = _grid(n, n)
    lab[(lab == 2) & (y < n / 2)] = 1
    return Workload(f"stratified_lens_{n}", n, n, (sigma_rg, sigma_rb, sigma_gb), (tau, tau, tau),
                    rho=rho_from_labels(lab), steps=steps)


def janus_droplet(n: int, Rr: float, Rg: float, Rb: float, drg: float, dgb: float, sigma,
                  tau: float = 0.8, y0: float = None, steps: int = 0) -> Workload:
    """General Janus droplet of fluids 0 (r) and 1 (g) in fluid 2 (b) on an n x n periodic
    lattice, laid out from its equilibrium geometry: the gb interface a circle of radius Rg
    centred at (xc, y0), the rb interface radius Rr at (xc, y0 + drg), the rg interface radius
    Rb at (xc, y0 + dgb), xc = (n - 1) / 2.  Fluid 0 fills the inside of both the rb and rg
    circles, fluid 1 the inside of the gb circle outside the rg circle."""
    xc = (n - 1) / 2.0
    y0 = Rg + 9.0 if y0 is None else y0
    x, y = _grid(n, n)
    def inside(cy, R):
        return (x - xc) ** 2 + (y - cy) ** 2 <= R * R
    in_r, in_g, in_b = inside(y0 + drg, Rr), inside(y0, Rg), inside(y0 + dgb, Rb)
    lab = np.full((n, n), 2, dtype=np.int64)
    lab[in_g & ~in_b] = 1
    lab[in_r & in_b] = 0
    return Workload(f"janus_{n}_{drg:g}", n, n, tuple(sigma), (tau, tau, tau), rho=rho_from_labels(lab),
                    steps=steps, meta={"Rr": Rr, "Rg": Rg, "Rb": Rb, "drg": drg, "dgb": dgb, "y0": y0})


def kissing_droplets(n: int, R: float, d: float, sigma, tau: float = 0.8) -> Workload:
    """Two droplets of radius R, fluid 0 below and fluid 1 above the centre line
    y = (n - 1) / 2, centres d apart on the line x = (n - 1) / 2, in fluid 2 (the kissing
    layout of the near-critical states of Sec. 4).  Where the disks overlap (d < 2 R) the
    centre line splits them."""
    c = (n - 1) / 2.0
    x, y = _grid(n, n)
    lab = np.full((n, n), 2, dtype=np.int64)
    lab[((x - c) ** 2 + (y - (c - d / 2)) ** 2 <= R * R) & (y < c)] = 0
    lab[((x - c) ** 2 + (y - (c + d / 2)) ** 2 <= R * R) & (y >= c)] = 1
    return Workload(f"kissing_{n}_{d:g}", n, n, tuple(sigma), (tau, tau, tau), rho=rho_from_labels(lab),
                    meta={"R": R, "d": d, "y_mid": c})


def engulfed_droplet(n: int, Rr: float, Rg: float, sigma, tau: float = 0.8, d: float | None = None) -> Workload:
    """A disk of fluid 0 (radius Rr) over a disk of fluid 1 (radius Rg), centres d apart on the
    line x = (n - 1) / 2 (default Rg - Rr: internally tangent), in fluid 2: the critical
    engulfing layout of Sec. 4; with d > Rg - Rr fluid 0 pokes out of fluid 1 (near-critical
    partial engulfing)."""
    c = (n - 1) / 2.0
    d = Rg - Rr if d is None else d
    x, y = _grid(n, n)
    lab = np.full((n, n), 2, dtype=np.int64)
    lab[(x - c) ** 2 + (y - (c - d / 2)) ** 2 <= Rg * Rg] = 1
    lab[(x - c) ** 2 + (y - (c + d / 2)) ** 2 <= Rr * Rr] = 0
    return Workload(f"engulfed_{n}", n, n, tuple(sigma), (tau, tau, tau), rho=rho_from_labels(lab),
                    meta={"Rr": Rr, "Rg": Rg, "d": d})


def flat_layers(nx: int, ny: int, y_interfaces=(0.25, 0.75), fluids=(2, 0)) -> np.ndarray:
    """Two flat layers uniform in x: fluid fluids[1] for y in [y0*ny, y1*ny), fluids[0] elsewhere."""
    x, y = _grid(nx, ny)
    lab = np.full((ny, nx), fluids[0], dtype=np.int64)
    lab[(y >= y_interfaces[0] * ny) & (y < y_interfaces[1] * ny)] = fluids[1]
    return rho_from_labels(lab)


def taylor_green(nx: int, ny: int, U: float = 1e-3, mix=(1.0, 0.0, 0.0)):
    """Uniform composition ``mix`` (sums to 1) and the Taylor-Green vortex velocity
    u_x = -U cos(kx x) sin(ky y), u_y = U (kx/ky) sin(kx x) cos(ky y)."""
    x, y = _grid(nx, ny)
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    u = np.stack([-U * np.cos(kx * x) * np.sin(ky * y),
                  U * (kx / ky) * np.sin(kx * x) * np.cos(ky * y)])
    rho = np.stack([np.full((ny, nx), float(m)) for m in mix])
    return rho, u
