"""The comparison segregation laws of Sec. 2 (Eqs. 15-17) on the GPU, through the C ABI,
against the FP64 oracle: one step per launch, two steps per launch, each precision, and a
batch whose instances use different laws."""
import numpy as np
import pytest

import oracle
from analysis import arc_length, contact_length, engulfed_rb_arc, interface_points, kissing_chord, mixed_nodes
from paper_1808_08555_amd import inputs, lbm3

pytestmark = pytest.mark.gpu

LAWS = ["spencer", "leclaire", "constant"]
SIG, TAU = (0.011, 0.013, 0.017), (0.7, 1.0, 1.3)  # a Neumann triangle with distinct angles


def _gpu(nx, ny, rho, steps, law, sigma=SIG, tau=TAU, precision="fp64", tile=None, mode=0):
    L = lbm3.Lattice(nx, ny, sigma, tau, precision=precision, beta_law=law).init(rho)
    try:
        if tile:
            L.set_tile(*tile)
        if mode:
            L.set_steps_per_launch(mode)
        return L.step(steps).state()
    finally:
        L.close()


def _oracle(nx, ny, rho, steps, law, sigma=SIG, tau=TAU):
    p = oracle.Params(nx, ny, sigma, tau, beta_law=law)
    return oracle.run(p, oracle.init(p, rho), steps)


@pytest.mark.parametrize("law", LAWS)
def test_parity_two_droplets_64_1000_steps(law):
    """The tangent disks of the 64^2 case (triple junctions, where 0 < C_t < 1), 1000 steps:
    the total distribution to 1e-11, the coloured populations to 1e-9 (the round-off
    amplification of colour traces, as for the paper's law), and a result that differs
    from the paper's law (the switch acts)."""
    w = inputs.two_droplets_64()
    g = _gpu(64, 64, w.rho, 1000, law, w.sigma, w.tau)
    o = _oracle(64, 64, w.rho, 1000, law, w.sigma, w.tau)
    d_tot, d_col = float(np.abs(g.sum(0) - o.sum(0)).max()), float(np.abs(g - o).max())
    print(f"{law}: |df_i| {d_tot:.2e} |df_ik| {d_col:.2e}")
    assert d_tot <= 1e-11 and d_col <= 1e-9
    paper = _gpu(64, 64, w.rho, 1000, "paper", w.sigma, w.tau)
    assert np.abs(paper - g).max() > 1e-6


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("tile", [(64, 16), (256, 0)])
def test_parity_ragged_random_mixture(law, tile):
    """301 x 83 random mixtures (three fluids at most nodes: C_t both below and at its cap),
    several strips and ragged row segments, 12 steps, to 1e-11."""
    rho = inputs.random_mixture(301, 83, 9, tiny_fraction=0.05)
    g = _gpu(301, 83, rho, 12, law, tile=tile)
    o = _oracle(301, 83, rho, 12, law)
    assert np.abs(g - o).max() <= 1e-11


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("precision,rtol", [("fp32_storage", 2e-6), ("fp32", 2e-5)])
def test_parity_reduced_precision(law, precision, rtol):
    """As for the paper's law: a 48^2 double droplet, 10 steps, relative to max |f|."""
    w = inputs.double_droplet(48, 9.0, 1.0, 1.2, seed=4, steps=0)
    g = _gpu(48, 48, w.rho, 10, law, w.sigma, w.tau, precision=precision)
    o = _oracle(48, 48, w.rho, 10, law, w.sigma, w.tau)
    err = np.abs(g - o).max() / np.abs(o).max()
    print(law, precision, "max rel |df|:", err)
    assert err <= rtol


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_storage"])
def test_two_step_pass_equals_single_steps_bitwise(law, precision):
    nx, ny = 97, 130
    rho = inputs.random_mixture(nx, ny, 5, tiny_fraction=0.0)
    a = _gpu(nx, ny, rho, 12, law, precision=precision, tile=(64, 9), mode=1)
    b = _gpu(nx, ny, rho, 12, law, precision=precision, tile=(64, 9), mode=2)
    assert np.isfinite(a).all() and np.array_equal(a, b)


def test_batch_of_mixed_laws_matches_plain_lattices_bitwise():
    """Four instances, one per law, in one batch (double droplets of different sizes, so
    triple junctions): 40 steps (two graph launches), densities equal to each plain
    lattice run alone, and to the oracle."""
    sides = [40, 52, 33, 64]
    sizes = [(n, n) for n in sides]
    laws = ["paper"] + LAWS
    rhos = [inputs.double_droplet(n, n / 5.0, 1.0, 1.3, seed=30 + i, steps=0).rho for i, n in enumerate(sides)]
    ps = [lbm3.make_params(nx, ny, SIG, TAU, beta_law=law) for (nx, ny), law in zip(sizes, laws)]
    b = lbm3.lbm3_batch_create(ps)
    try:
        for i, rho in enumerate(rhos):
            lbm3.lbm3_batch_init_fields(b, i, rho)
        lbm3.lbm3_batch_step(b, 40)
        for i, ((nx, ny), law) in enumerate(zip(sizes, laws)):
            _, rho = lbm3.lbm3_batch_observables(b, i, nx, ny, want_rho=True)
            L = lbm3.Lattice(nx, ny, SIG, TAU, beta_law=law).init(rhos[i]).step(40)
            ref = L.densities()
            L.close()
            assert np.array_equal(rho, ref), law
            o = _oracle(nx, ny, rhos[i], 40, law)
            assert np.abs(rho - o.sum(axis=1)).max() <= 1e-11, law
    finally:
        lbm3.lbm3_batch_destroy(b)


def test_adjoint_refuses_other_laws():
    L = lbm3.Lattice(16, 16, SIG, TAU, beta_law="spencer").init(inputs.random_mixture(16, 16, 1))
    try:
        with pytest.raises(lbm3.Lbm3Error) as e:
            lbm3.lbm3_adjoint_record(L.h, 2, 1)
        assert e.value.code == lbm3.LBM3_EUNSUPPORTED
    finally:
        L.close()


def _run(w, law, steps):
    L = lbm3.Lattice(w.nx, w.ny, w.sigma, w.tau, beta_law=law).init(w.rho)
    try:
        obs, rho, _ = L.step(steps).observables(want_rho=True)
        assert obs["nonfinite"] == 0
        return rho
    finally:
        L.close()


def test_critical_kissing_state_paper_law_against_the_comparison_laws():
    """Sec. 4, near-critical and critical states: two R = 60 droplets (fluids 0, 1) touching
    in fluid 2 on 300^2, sigma_rg = 0.01 = sigma_rb + sigma_gb (critical, the kissing
    state), nu = 0.1, 20000 steps.  The paper's law keeps a point contact (only the
    diffuse tails, about 9 nodes); with the constant beta of Eq. (17) the droplets form a
    flat contact about 50 nodes long; Eq. (16) has no triangle here and gives the constant
    law's result (the paper reports the two as almost the same)."""
    w = inputs.kissing_droplets(300, 60.0, 120.0, (0.01, 0.005, 0.005))
    res = {law: _run(w, law, 20000) for law in ("paper", "constant", "leclaire")}
    Lc = {law: contact_length(r, w.meta["y_mid"]) for law, r in res.items()}
    print("contact length L_rg:", Lc)
    assert Lc["paper"] < 0.25 * Lc["constant"]
    assert np.array_equal(res["leclaire"], res["constant"])


def test_critical_engulfing_state_paper_law_against_the_constant_law():
    """Sec. 4, critical engulfing: a fluid-0 disk (R_r = 60) inside a fluid-1 disk (R_g = 80),
    internally tangent, in fluid 2, sigma_rg = sigma_gb = 0.01, sigma_rb = 0.02 (critical:
    complete engulfing, no rb interface), 50000 steps.  With the paper's law the rb
    interface shrinks to a few mixed nodes; with the constant beta of Eq. (17) fluid 0
    stays exposed to fluid 2 along an arc (hundreds of mixed nodes)."""
    w = inputs.engulfed_droplet(300, 60.0, 80.0, (0.01, 0.02, 0.01))
    n = {law: mixed_nodes(_run(w, law, 50000), 0, 2) for law in ("paper", "constant")}
    print("rb mixed nodes:", n)
    assert n["paper"] < 0.15 * n["constant"] and n["constant"] > 200


def test_near_critical_kissing_sweep_interface_length():
    """Sec. 4, kissing and near-kissing states with the paper's law: two R = 60 droplets,
    sigma_rg = 0.01, sigma_gb = sigma_rb from 0.0046 to 0.0058 in steps of 2e-4, laid out at
    their analytic distance d_rg (Eq. drg), nu = 0.1, 50 000 steps (the lengths are steady from
    20 000 on).  L_rg is measured as the contact across the centre line (sum of 1 - c_b over
    the two rows beside it, analysis.contact_length) and as the extent of the rg interface
    (points where c_0 = c_1 with c_b < 0.05).  At and below the kissing state (analytic
    L_rg = 0) the droplets keep a point contact: no rg interface, only the diffuse tails
    (contact <= 12).  From 0.0054 on the contact is the analytic chord plus the diffuse ends,
    within 8 nodes (measured +2.4 to +5.9).  At 0.0052 (analytic chord 33) the model keeps a
    point contact too (contact 17, no rg interface): reported, not asserted.  The comparison
    law of Eq. (17) forms a flat contact of 35-50 nodes where the analytic one is 0."""
    res = []
    for sgb in (0.0046, 0.0048, 0.005, 0.0052, 0.0054, 0.0056, 0.0058):
        L_an = kissing_chord(60.0, 0.01, sgb)
        d = 120.0 if sgb <= 0.005 else 60.0 * 0.01 / sgb
        w = inputs.kissing_droplets(300, 60.0, d, (0.01, sgb, sgb))
        laws = ("paper", "constant") if sgb <= 0.005 else ("paper",)
        for law in laws:
            rho = _run(w, law, 50000)
            c = rho / rho.sum(0)
            pts = interface_points(c, 0, 1)
            ext = float(pts[:, 0].max() - pts[:, 0].min()) if len(pts) else 0.0
            res.append((sgb, law, L_an, contact_length(rho, w.meta["y_mid"]), ext))
    for r in res:
        print("sigma_gb %.4f %-8s analytic %5.1f contact %5.1f rg extent %5.1f" % r)
    for sgb, law, L_an, cl, ext in res:
        if law == "constant":
            assert cl > 30.0, (sgb, cl)
        elif sgb <= 0.005:
            assert cl <= 12.0 and ext == 0.0, (sgb, cl, ext)
        elif sgb >= 0.0054:
            assert abs(cl - L_an) <= 8.0 and ext > 0.5 * L_an, (sgb, cl, L_an, ext)


def test_near_critical_engulfing_sweep_interface_length():
    """Sec. 4, critical and near-critical engulfing with the paper's law: a fluid-0 droplet
    (R_r = 60) partly engulfed by a fluid-1 droplet (R_g = 80), sigma_rg = sigma_gb = 0.01,
    sigma_rb from 0.0194 to 0.0204 in steps of 2e-4, laid out with its centres at the analytic
    distance d_rg, nu = 0.1, 100 000 steps.  L_rb, the length of fluid 0's arc exposed to fluid
    2, is measured on the rb interface points (analysis.arc_length).  At and beyond the
    critical state (analytic L_rb = 0) the exposure vanishes: no rb interface and at most a few
    mixed nodes.  Below it the model engulfs more than the analytic geometry: L_rb = 72 against
    100 at 0.0194, and at 0.0196 and 0.0198 the exposed arc keeps shrinking toward complete
    engulfing (analytic 86 and 64): reported, only the ordering is asserted.  The constant law
    of Eq. (17) leaves an exposed arc of 170-190 nodes at the critical and supercritical
    states."""
    res = []
    for srb in (0.0194, 0.0196, 0.0198, 0.02, 0.0202, 0.0204):
        d, L_an = engulfed_rb_arc(60.0, 80.0, srb, 0.01)
        w = inputs.engulfed_droplet(300, 60.0, 80.0, (0.01, srb, 0.01), d=d)
        laws = ("paper", "constant") if srb >= 0.02 else ("paper",)
        for law in laws:
            rho = _run(w, law, 100000)
            c = rho / rho.sum(0)
            res.append((srb, law, L_an, arc_length(interface_points(c, 0, 2)), mixed_nodes(rho, 0, 2)))
    for r in res:
        print("sigma_rb %.4f %-8s analytic %5.1f rb arc %6.1f mixed nodes %4d" % r)
    paper = {r[0]: r for r in res if r[1] == "paper"}
    for srb, law, L_an, arc, mix in res:
        if law == "constant":
            assert arc > 120.0, (srb, arc)
        elif srb >= 0.02:
            assert arc == 0.0 and mix <= 10, (srb, arc, mix)
    assert paper[0.0194][3] > 50.0 and paper[0.0194][3] > paper[0.0196][3] >= paper[0.0198][3]
