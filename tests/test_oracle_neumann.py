"""Neumann-triangle geometry of Sec. 4 against the values the paper prints: the lens of a
droplet spreading between two stratified fluids (Eq. 23, Table 3) and the general Janus
droplet (Eqs. gjd_01-06, Table 4), each with the oracle's Neumann-triangle cosines of
Eq. (14) (tests/golden/table3_lens.json, tests/golden/table4_gjd.json)."""
import json
import math
import os

import pytest

import oracle
from analysis import gjd_geometry, lens_analytic

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table3_lens.json")))
GJD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table4_gjd.json")))


def _angles(case):
    c = GOLDEN["cases"][case]
    p = oracle.Params(8, 8, (c["sigma_rg"], c["sigma_rb"], GOLDEN["setup"]["sigma_gb"]))
    return math.acos(oracle.X(p, 0, 1)), math.acos(oracle.X(p, 0, 2))


@pytest.mark.parametrize("case", sorted(GOLDEN["cases"]))
def test_table3_analytic_columns(case):
    """The four cases are lenses with contact angles of 30, 60 or 90 degrees, their
    tensions printed to two or three digits (0.0087 for 0.01 sin 60 ...).  The printed
    analytic columns follow the round angles: the oracle's angles from the printed tensions
    lie within 0.75 degrees of a multiple of 30; with those multiples and A = pi R^2 the
    columns agree to 0.3 %, and with the oracle's own angles to 2 %.  A swapped pair of
    contact angles or a wrong Eq. (23) misses by far more (case b: h1 8.7 vs h2 18.8)."""
    c = GOLDEN["cases"][case]
    t1, t2 = _angles(case)
    r1, r2 = (30 * round(math.degrees(t) / 30) for t in (t1, t2))
    assert abs(math.degrees(t1) - r1) < 0.75 and abs(math.degrees(t2) - r2) < 0.75
    A = math.pi * GOLDEN["setup"]["R"] ** 2
    printed = (c["D_a"], c["h1_a"], c["h2_a"])
    whole = lens_analytic(math.radians(r1), math.radians(r2), A)
    own = lens_analytic(t1, t2, A)
    for got, want in zip(whole, printed):
        assert abs(got / want - 1) < 3e-3, (case, whole, printed)
    for got, want in zip(own, printed):
        assert abs(got / want - 1) < 2e-2, (case, own, printed)


@pytest.mark.parametrize("row", GJD["rows"], ids=lambda r: f"drg{r['d_rg']}")
def test_table4_general_janus_geometry(row):
    """Eqs. (gjd_01)-(gjd_06) from R_r, R_g, R_b and d_rg reproduce Table 4's sigma_gb,
    sigma_rb (printed to 1e-5) and d_gb (to 0.01); and the oracle's Neumann angles from
    Table 4's tensions equal the geometric phi_kl to 0.25 degree (the tensions are printed
    to three digits, which moves phi_rg = 117 degrees by 0.16)."""
    s = GJD["setup"]
    g = gjd_geometry(s["Rr"], s["Rg"], s["Rb"], row["d_rg"], s["sigma_rg"])
    assert abs(g["sigma_gb"] - row["sigma_gb"]) <= 1e-5
    assert abs(g["sigma_rb"] - row["sigma_rb"]) <= 1e-5
    assert abs(g["d_gb"] - row["d_gb"]) <= 0.01
    p = oracle.Params(8, 8, (s["sigma_rg"], row["sigma_rb"], row["sigma_gb"]))
    for (k, l), name in (((0, 1), "phi_rg"), ((0, 2), "phi_rb"), ((1, 2), "phi_gb")):
        assert abs(math.degrees(math.acos(oracle.X(p, k, l)) - g[name])) < 0.25, (name, row)


@pytest.mark.parametrize("row", GJD["rows"], ids=lambda r: f"drg{r['d_rg']}")
def test_table4_layout_pressure_balance(row):
    """An equilibrium of three circular arcs needs consistent pressure jumps (Young-Laplace
    on each arc, Eq. 26): sigma_rg / R_b = sigma_rb / R_r - sigma_gb / R_g.  The rows with
    d_rg >= 60 (angles from Eq. gjd_05) satisfy it to 0.2 %; the row d_rg = 40 (Eq. gjd_04)
    misses by 41 %, so its layout is not an equilibrium (the GPU test leaves it out)."""
    s = GJD["setup"]
    lhs = s["sigma_rg"] / s["Rb"]
    rhs = row["sigma_rb"] / s["Rr"] - row["sigma_gb"] / s["Rg"]
    if row["d_rg"] >= 60:
        assert abs(rhs / lhs - 1) < 2e-3
    else:
        assert abs(rhs / lhs - 1) > 0.3


PJD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table5_pjd.json")))


@pytest.mark.parametrize("row", PJD["rows"], ids=lambda r: f"f{r['fraction']}")
def test_table5_perfect_janus_geometry(row):
    """Eq. (pjd) for R = 80 reproduces Table 5's R_b and d_gb (printed to 0.01).  The solution
    is checked against the geometry it describes, not only the printed numbers: the rg arc
    meets the droplet's circle at a right angle (R^2 + R_b^2 = d_gb^2, which the zero rg
    tension requires: the matrix angle at the junction is 180 degrees and the red and green
    ones 90), and the area of the disk inside the rg circle, counted on a fine grid, is the
    requested fraction of the disk."""
    import numpy as np
    from analysis import pjd_geometry
    R = PJD["setup"]["R"]
    g = pjd_geometry(row["fraction"], R)
    assert abs(g["R_b"] - row["R_b"]) <= 0.01 and abs(g["d_gb"] - row["d_gb"]) <= 0.01
    assert abs(R * R + g["R_b"] ** 2 - g["d_gb"] ** 2) < 1e-9 * g["d_gb"] ** 2
    h = R / 1000.0
    y, x = np.mgrid[-R + h / 2:R:h, -R + h / 2:R:h]
    disk = x * x + y * y <= R * R
    cap = disk & (x * x + (y - g["d_gb"]) ** 2 <= g["R_b"] ** 2)
    assert abs(cap.sum() / disk.sum() - row["fraction"]) < 2e-4


def test_perfect_janus_tensions_are_the_degenerate_neumann_limit():
    """With sigma_rg = 1e-8 and sigma_rb = sigma_gb = 0.01 the oracle's Neumann cosines
    (Eq. 14) put the matrix angle at the junction at 180 degrees (X_rg within 1e-12 of 1,
    taken as exactly 1) and the red and green angles at 90 degrees (X_rb = X_gb ~ 5e-7)."""
    s = PJD["setup"]
    p = oracle.Params(8, 8, (s["sigma_rg"], s["sigma_rb"], s["sigma_gb"]))
    assert 1 - oracle.X(p, 0, 1) < 1e-12 and oracle.g(oracle.X(p, 0, 1)) == -1.0
    for k, l in ((0, 2), (1, 2)):
        assert abs(math.degrees(math.acos(oracle.X(p, k, l))) - 90.0) < 1e-3
