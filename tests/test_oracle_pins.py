"""The oracle against what the paper and the mathematics fix (CPU only)."""
import math

import numpy as np
import pytest

import oracle
import oracle_pins as P
from paper_1808_08555_amd import inputs


@pytest.mark.parametrize("pin", P.FAST_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


def test_pin_interface_constant_k():
    P.pin_interface_constant_k()


def test_pin_conservation():
    P.pin_conservation()


def test_compound_droplet_laplace_error():
    """Compound droplet (Sec. 3.2): eq. (27)'s error with R from the conserved colour areas
    is inside the band the paper prints in Table 1 (0.57 %..1.3 % for R_r = 30..15 at
    R_g = 2 R_r); here R_r = 12 on 96^2, so the bound is the table's 1.3 %.  The spurious
    velocity is of the order of Table 2's present-model value (1.7e-5)."""
    n, rr = 96, 12.0
    w = inputs.compound_droplet(n, rr, 2 * rr, 0.01, 0.01, 0.01, steps=6000)
    p = oracle.Params(n, n, w.sigma, w.tau)
    f = oracle.run(p, oracle.init(p, w.rho), w.steps)
    rho, u, _, _ = oracle.fields(p, f)
    c = rho / rho.sum(0)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    r = np.sqrt((x - w.meta["centre"]) ** 2 + (y - w.meta["centre"]) ** 2)
    Rr = math.sqrt(c[0].sum() / math.pi)
    Rg = math.sqrt((c[0] + c[1]).sum() / math.pi)
    pr = rho.sum(0) / 3
    p_in = pr[r <= Rr / 2].mean()
    p_sh = pr[np.abs(r - (Rr + Rg) / 2) <= (Rg - Rr) / 4].mean()
    p_out = pr[r >= Rg + 10].mean()
    eps = abs((p_sh - p_out) * Rg + (p_in - p_sh) * Rr - 0.02) / 0.02
    assert eps < 0.013, eps
    umax = np.sqrt((u ** 2).sum(0)).max()
    assert 3e-6 < umax < 1e-4, umax


def test_double_bubble_two_droplets_64():
    """The 64^2 two-droplet case has its disks touching, so with equal tensions they join
    into a symmetric double bubble: the shared interface is flat and each lobe is a circle of
    radius R_a cut by a chord at R_a/2 from its centre (120-degree junctions), area
    R_a^2 (2 pi/3 + sqrt(3)/4); its pressure jump is sigma/R_a."""
    w = inputs.two_droplets_64()
    p = oracle.Params(w.nx, w.ny, w.sigma, w.tau)
    f = oracle.run(p, oracle.init(p, w.rho), 2000)
    rho, _, _, _ = oracle.fields(p, f)
    c = rho / rho.sum(0)
    pr = rho.sum(0) / 3
    p_out = pr[c[2] > 0.999].mean()
    for k in (0, 1):
        Ra = math.sqrt(c[k].sum() / (2 * math.pi / 3 + math.sqrt(3) / 4))
        dp = pr[c[k] > 0.99].mean() - p_out
        assert abs(dp / (0.01 / Ra) - 1) < 0.06, (k, dp, 0.01 / Ra)
    # the two lobes mirror each other about x = 32 (up to the tie-break node at (32, 32))
    assert abs(c[0].sum() - c[1].sum()) < 2.0
