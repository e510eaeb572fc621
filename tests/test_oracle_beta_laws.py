"""The comparison segregation laws of Sec. 2 (Eqs. 15-17) in the oracle, pinned to the
geometry of the Neumann triangle and to closed forms, and the host constants the library
derives for them (lbm3_derived, no GPU) against the oracle.

The triangle angles here come from coordinates (atan2 of the edge vectors), not from the
law of cosines the oracle uses, so a swapped pair, sign or angle fails."""
import math

import numpy as np
import pytest

import oracle
from paper_1808_08555_amd import lbm3

B0 = 0.7
PAIRS = [(0, 1), (0, 2), (1, 2)]  # rg, rb, gb


def triangle_angles(s_rg, s_rb, s_gb):
    """Interior angles opposite the sides (phi_rg, phi_rb, phi_gb) of the triangle with side
    lengths sigma: P = (0, 0), Q = (s_rg, 0), R with |PR| = s_rb, |QR| = s_gb."""
    x = (s_rg ** 2 + s_rb ** 2 - s_gb ** 2) / (2 * s_rg)
    R = np.array([x, math.sqrt(s_rb ** 2 - x ** 2)])
    P, Q = np.zeros(2), np.array([s_rg, 0.0])

    def ang(o, a, b):
        u, v = a - o, b - o
        return abs(math.atan2(u[0] * v[1] - u[1] * v[0], u @ v))

    # the angle at R faces PQ (sigma_rg), at Q faces PR (sigma_rb), at P faces QR (sigma_gb)
    return ang(R, P, Q), ang(Q, P, R), ang(P, Q, R)


def P3(rho):
    r = sum(rho)
    return rho[0] * rho[1] * rho[2] / r ** 3


def ct(rho):
    return min(35 * P3(rho), 1.0)


RHOS = [(0.4, 0.35, 0.25), (0.9, 0.05, 0.05), (0.34, 0.33, 0.33), (0.6, 0.3, 0.1), (0.2, 0.7, 0.1)]


def test_triangle_helper_is_a_triangle():
    a = triangle_angles(0.01, 0.012, 0.014)
    assert abs(sum(a) - math.pi) < 1e-14
    assert a[2] > a[1] > a[0]  # the largest side faces the largest angle


@pytest.mark.parametrize("law", ["spencer", "leclaire", "constant", "paper"])
def test_two_fluid_nodes_take_beta0(law):
    """Where only two fluids are present every law gives beta^0 (the density factor is 0)."""
    p = oracle.Params(4, 4, (0.01, 0.013, 0.008), beta_law=law)
    for rho in [(0.6, 0.4, 0.0), (0.0, 0.3, 0.7), (0.5, 0.0, 0.5)]:
        for k, l in PAIRS:
            assert oracle.beta(p, k, l, rho) == B0


def test_constant_law_is_beta0_everywhere():
    """Eq. (17)."""
    p = oracle.Params(4, 4, (0.01, 0.03, 0.012), beta_law="constant")
    for rho in RHOS:
        for k, l in PAIRS:
            assert oracle.beta(p, k, l, rho) == B0
            assert oracle.beta(p, l, k, rho) == B0


@pytest.mark.parametrize("sig", [(0.01, 0.012, 0.014), (0.014, 0.01, 0.012), (0.012, 0.014, 0.01),
                                 (0.01, 0.01, 0.01), (0.005, 0.009, 0.006)])
def test_spencer_against_triangle_geometry(sig):
    """Eq. (15) as printed: beta_rg = beta0, beta_rb uses sin(phi_gb), beta_gb uses
    sin(phi_rb), with the factor 27 rho_r rho_g rho_b / rho^3."""
    phi_rg, phi_rb, phi_gb = triangle_angles(*sig)
    p = oracle.Params(4, 4, sig, beta_law="spencer")
    for rho in RHOS:
        s = 27 * P3(rho)
        want = [B0, B0 * (1 + s * (math.sin(phi_gb) - 1)), B0 * (1 + s * (math.sin(phi_rb) - 1))]
        for q, (k, l) in enumerate(PAIRS):
            assert abs(oracle.beta(p, k, l, rho) - want[q]) < 1e-14
            assert oracle.beta(p, l, k, rho) == oracle.beta(p, k, l, rho)


def test_spencer_equilateral_closed_form():
    p = oracle.Params(4, 4, (0.01, 0.01, 0.01), beta_law="spencer")
    rho = (1 / 3, 1 / 3, 1 / 3)  # 27 rho_r rho_g rho_b / rho^3 = 1
    assert oracle.beta(p, 0, 1, rho) == B0
    for k, l in [(0, 2), (1, 2)]:
        assert abs(oracle.beta(p, k, l, rho) - B0 * math.sqrt(3) / 2) < 1e-15


@pytest.mark.parametrize("sig", [(0.01, 0.012, 0.014), (0.014, 0.01, 0.012), (0.012, 0.014, 0.01),
                                 (0.005, 0.009, 0.006), (0.02, 0.011, 0.012)])
def test_leclaire_against_triangle_geometry(sig):
    """Eq. (16): beta0 for the pair of the largest angle, beta0 + beta0 C_t [sin(pi - phi_max
    - phi_kl) - 1] (the sine of the third angle) for the other two."""
    phis = triangle_angles(*sig)
    qmax = int(np.argmax(phis))
    p = oracle.Params(4, 4, sig, beta_law="leclaire")
    for rho in RHOS:
        for q, (k, l) in enumerate(PAIRS):
            if q == qmax:
                want = B0
            else:
                third = [a for i, a in enumerate(phis) if i not in (q, qmax)][0]
                want = B0 + B0 * ct(rho) * (math.sin(third) - 1)
            assert abs(oracle.beta(p, k, l, rho) - want) < 1e-14, (sig, rho, q)


def test_leclaire_degrades_to_spencer_when_phi_rg_is_largest():
    """With phi_max = phi_rg the two laws share beta_rg = beta0 and the sines of beta_rb and
    beta_gb; they differ only in the density factor (C_t against 27 rho_r rho_g rho_b/rho^3)."""
    sig = (0.02, 0.011, 0.012)
    assert np.argmax(triangle_angles(*sig)) == 0
    pl = oracle.Params(4, 4, sig, beta_law="leclaire")
    ps = oracle.Params(4, 4, sig, beta_law="spencer")
    for rho in RHOS:
        assert oracle.beta(pl, 0, 1, rho) == B0 == oracle.beta(ps, 0, 1, rho)
        for k, l in [(0, 2), (1, 2)]:
            hl = (oracle.beta(pl, k, l, rho) - B0) / (B0 * ct(rho))
            hs = (oracle.beta(ps, k, l, rho) - B0) / (B0 * 27 * P3(rho))
            assert abs(hl - hs) < 1e-13


def test_leclaire_equal_angles_take_the_first_pair():
    """Reading: on equal maxima the first pair in the order rg, rb, gb keeps beta0."""
    p = oracle.Params(4, 4, (0.01, 0.01, 0.01), beta_law="leclaire")
    rho = (0.4, 0.35, 0.25)
    assert oracle.beta(p, 0, 1, rho) == B0
    for k, l in [(0, 2), (1, 2)]:
        assert abs(oracle.beta(p, k, l, rho) - (B0 + B0 * ct(rho) * (math.sqrt(3) / 2 - 1))) < 1e-15


@pytest.mark.parametrize("sig", [(0.005, 0.02, 0.01), (0.01, 0.015, 0.005), (0.03, 0.01, 0.01)])
def test_leclaire_without_a_triangle_is_beta0(sig):
    """No Neumann triangle (one tension at or above the sum of the other two, the critical
    states included): beta_kl = beta0."""
    p = oracle.Params(4, 4, sig, beta_law="leclaire")
    for rho in RHOS:
        for k, l in PAIRS:
            assert oracle.beta(p, k, l, rho) == B0


def test_spencer_without_a_triangle_clamps_the_angles():
    """Reading: cos(phi) of Eq. (14) clamped to [-1, 1], so sin(phi) = 0 and beta_rb, beta_gb
    = beta0 (1 - 27 rho_r rho_g rho_b / rho^3)."""
    p = oracle.Params(4, 4, (0.005, 0.02, 0.01), beta_law="spencer")
    for rho in RHOS:
        assert oracle.beta(p, 0, 1, rho) == B0
        for k, l in [(0, 2), (1, 2)]:
            assert abs(oracle.beta(p, k, l, rho) - B0 * (1 - 27 * P3(rho))) < 1e-15


@pytest.mark.parametrize("law", ["spencer", "leclaire", "constant"])
def test_library_constants_of_each_law_match_the_oracle(law):
    """The library's host precompute (beta_kl = beta0 (1 + s g_kl), s = min(c P, 1) with
    c = 27 for Spencer, 35 otherwise) gives the oracle's beta_kl at every node density."""
    rng = np.random.default_rng(17)
    sets = [tuple(rng.uniform(0.004, 0.02, 3)) for _ in range(12)]
    sets += [(0.01, 0.01, 0.01), (0.005, 0.015, 0.01), (0.005, 0.02, 0.01)]
    for sig in sets:
        _, g, _ = lbm3.lbm3_derived(lbm3.make_params(8, 8, sig, beta_law=law))
        p = oracle.Params(4, 4, sig, beta_law=law)
        for rho in RHOS:
            s = min((27 if law == "spencer" else 35) * P3(rho), 1.0)
            for q, (k, l) in enumerate(PAIRS):
                assert abs(B0 * (1 + s * g[q]) - oracle.beta(p, k, l, rho)) < 1e-14, (law, sig, q)


def test_library_rejects_an_unknown_law():
    import ctypes
    p = lbm3.make_params(8, 8, beta_law=4)
    h = ctypes.c_void_p()
    assert lbm3.lib().lbm3_create(ctypes.byref(p), None, ctypes.byref(h)) == lbm3.LBM3_EINVAL
    assert "beta_law" in lbm3.lbm3_last_error()


# ---- planted mistakes in a copy of the oracle source (CPU): each must fail a pin above
def _pins():
    sets = [(0.01, 0.012, 0.014), (0.014, 0.01, 0.012), (0.012, 0.014, 0.01), (0.02, 0.011, 0.012)]
    yield from (lambda s=s: test_spencer_against_triangle_geometry(s) for s in sets)
    yield test_spencer_equilateral_closed_form
    yield from (lambda s=s: test_leclaire_against_triangle_geometry(s) for s in sets)
    yield test_leclaire_equal_angles_take_the_first_pair
    yield from (lambda s=s: test_leclaire_without_a_triangle_is_beta0(s)
                for s in [(0.005, 0.02, 0.01), (0.01, 0.015, 0.005)])
    yield test_spencer_without_a_triangle_clamps_the_angles
    yield test_constant_law_is_beta0_everywhere


LAW_MUTANTS = {
    "spencer_sines_swapped": ("return p->beta0 * (1.0 + s * (sin(neumann_phi(p, 1, 2)) - 1.0));",
                              "return p->beta0 * (1.0 + s * (sin(neumann_phi(p, 0, 2)) - 1.0));"),
    "spencer_factor_35": ("double s = 27.0 * rho[0]", "double s = 35.0 * rho[0]"),
    "leclaire_max_pair_not_kept": ("if (k == kmax && l == lmax) return p->beta0;", ""),
    "leclaire_angle_sum": ("sin(ORACLE_PI - phimax - neumann_phi(p, k, l))", "sin(phimax - neumann_phi(p, k, l))"),
    "leclaire_smallest_angle": ("if (ph > phimax) {", "if (ph < phimax) {"),
    "leclaire_ties_to_last": ("if (ph > phimax) {", "if (ph >= phimax) {"),
    "leclaire_no_fallback": ("if (!neumann_triangle_exists(p)) return p->beta0;", ""),
    "beta_not_symmetric": ("    if (k > l) {\n        int t = k;\n        k = l;\n        l = t;\n    }\n", ""),
    "constant_law_missing": ("if (p->beta_law == 3) return p->beta0; /* Eq. (17) */", ""),
}


@pytest.mark.parametrize("name", sorted(LAW_MUTANTS))
def test_planted_mistake_in_a_comparison_law_is_caught(name, tmp_path):
    import os
    old, new = LAW_MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, f"pattern for {name} must occur exactly once"
    so = oracle.compile_source(src.replace(old, new), os.path.join(tmp_path, f"mut_{name}.so"))
    caught = None
    with oracle.use_library(so):
        for pin in _pins():
            try:
                pin()
            except AssertionError as e:
                caught = e
                break
    assert caught is not None, f"no pin catches the planted mistake {name}"
