"""The lens of Sec. 4 (a droplet spreading between two stratified fluids): the analytic
lens geometry of Eq. (23), with contact angles theta_1 = phi_rg and theta_2 = phi_rb from
the oracle's Neumann-triangle cosines (Eq. 14), against the analytic columns printed in
Table 3 (tests/golden/table3_lens.json)."""
import json
import math
import os

import pytest

import oracle
from analysis import lens_analytic

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table3_lens.json")))


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
