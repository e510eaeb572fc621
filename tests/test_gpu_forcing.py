"""The comparison forcing (the perturbation operator of Eqs. 4-5) on the GPU through the C
ABI: parity with the FP64 oracle, every launch form (two steps per launch and the batch
bitwise equal to single steps), the adjoint's refusal, and the comparison of Table 2 (the
paper's forcing gives the smaller spurious velocities; the perturbation row reproduced)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1808_08555_amd import inputs, lbm3

from analysis import compound_laplace

pytestmark = pytest.mark.gpu

SIG, TAU = (0.011, 0.013, 0.017), (0.7, 1.0, 1.3)
PT = "perturbation"


def _gpu(nx, ny, rho, steps, sigma=SIG, tau=TAU, precision="fp64", tile=None, law="paper"):
    L = lbm3.Lattice(nx, ny, sigma, tau, precision=precision, forcing=PT, beta_law=law).init(rho)
    try:
        if tile:
            L.set_tile(*tile)
        return L.step(steps).state()
    finally:
        L.close()


def _oracle(nx, ny, rho, steps, sigma=SIG, tau=TAU, law="paper"):
    p = oracle.Params(nx, ny, sigma, tau, forcing=PT, beta_law=law)
    return oracle.run(p, oracle.init(p, rho), steps)


def test_parity_two_droplets_64_1000_steps():
    """As for the paper's forcing: the total distribution to 1e-11 after 1000 steps, the
    coloured populations to 1e-9; and a result different from Guo forcing."""
    w = inputs.two_droplets_64()
    g = _gpu(64, 64, w.rho, 1000, w.sigma, w.tau)
    o = _oracle(64, 64, w.rho, 1000, w.sigma, w.tau)
    d_tot, d_col = float(np.abs(g.sum(0) - o.sum(0)).max()), float(np.abs(g - o).max())
    print(f"perturbation: |df_i| {d_tot:.2e} |df_ik| {d_col:.2e}")
    assert d_tot <= 1e-11 and d_col <= 1e-9
    L = lbm3.Lattice(64, 64, w.sigma, w.tau).init(w.rho)
    guo = L.step(1000).state()
    L.close()
    assert np.abs(guo - g).max() > 1e-6


@pytest.mark.parametrize("tile", [(64, 16), (128, 7), (256, 0), (512, 0)])
def test_parity_ragged_random_mixture(tile):
    rho = inputs.random_mixture(301, 83, 9, tiny_fraction=0.05)
    assert np.abs(_gpu(301, 83, rho, 12, tile=tile) - _oracle(301, 83, rho, 12)).max() <= 1e-11


def test_parity_with_a_comparison_law():
    rho = inputs.random_mixture(97, 61, 2, tiny_fraction=0.05)
    g = _gpu(97, 61, rho, 12, law="leclaire")
    assert np.abs(g - _oracle(97, 61, rho, 12, law="leclaire")).max() <= 1e-11


@pytest.mark.parametrize("nx,ny", [(1, 5), (3, 2), (5, 7)])
def test_parity_degenerate_lattices(nx, ny):
    rho = inputs.random_mixture(nx, ny, 21, tiny_fraction=0.0)
    assert np.abs(_gpu(nx, ny, rho, 5) - _oracle(nx, ny, rho, 5)).max() <= 1e-11


@pytest.mark.parametrize("precision,rtol", [("fp32_storage", 2e-6), ("fp32", 2e-5)])
def test_parity_reduced_precision(precision, rtol):
    w = inputs.double_droplet(48, 9.0, 1.0, 1.2, seed=4, steps=0)
    g = _gpu(48, 48, w.rho, 10, w.sigma, w.tau, precision=precision)
    o = _oracle(48, 48, w.rho, 10, w.sigma, w.tau)
    err = np.abs(g - o).max() / np.abs(o).max()
    print(precision, "max rel |df|:", err)
    assert err <= rtol


def test_observables_use_the_force_free_velocity():
    """u_max, momentum and kinetic energy with u = sum_i f_i e_i / rho, against the oracle."""
    w = inputs.two_droplets_64()
    L = lbm3.Lattice(64, 64, w.sigma, w.tau, forcing=PT).init(w.rho).step(300)
    obs, _, f = L.observables(want_f=True)
    L.close()
    p = oracle.Params(64, 64, w.sigma, w.tau, forcing=PT)
    ref = oracle.observables(p, f)
    print(obs, ref)
    assert np.abs(obs["momentum"] - ref["momentum"]).max() < 1e-12
    assert abs(obs["kinetic_energy"] / ref["kinetic_energy"] - 1) < 1e-9
    assert abs(obs["u_max"] / ref["u_max"] - 1) < 1e-9


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_storage"])
def test_two_step_pass_equals_single_steps_bitwise(precision):
    nx, ny = 97, 130
    rho = inputs.random_mixture(nx, ny, 5, tiny_fraction=0.0)
    out = []
    for mode in (1, 2):
        L = lbm3.Lattice(nx, ny, SIG, TAU, precision=precision, forcing=PT).init(rho)
        L.set_tile(64, 9)
        L.set_steps_per_launch(mode)
        assert lbm3.lbm3_get_pair_launch(L.h)[0] == mode
        out.append(L.step(12).state())
        L.close()
    assert np.isfinite(out[0]).all() and np.array_equal(out[0], out[1])


def test_full_size_default_launch_pairs_and_matches_the_oracle_on_sampled_nodes():
    """1024 x 512 (2^19 nodes, two steps per launch by default): 21 steps (ten two-step
    launches after the first single step), then one more step compared with the oracle's
    node-local step at sampled nodes, to 1e-11."""
    nx, ny = 1024, 512
    w = inputs.double_droplet(512, 60.0, 1.0, 1.3, seed=8, steps=0)
    rho = np.concatenate([w.rho, w.rho], axis=2)
    L = lbm3.Lattice(nx, ny, SIG, TAU, forcing=PT).init(rho)
    try:
        assert lbm3.lbm3_get_pair_launch(L.h)[0] == 2
        fa = L.step(21).state()
        fb = L.step(1).state()
    finally:
        L.close()
    rng = np.random.default_rng(3)
    xs = np.concatenate([[0, nx - 1, 511, 512], rng.integers(0, nx, 80)])
    ys = np.concatenate([[0, ny - 1, 255, 256], rng.integers(0, ny, 80)])
    p = oracle.Params(nx, ny, SIG, TAU, forcing=PT)
    o = oracle.step_nodes(p, fa, xs, ys)
    assert np.abs(fb[:, :, ys, xs].transpose(2, 0, 1) - o).max() <= 1e-11


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_plain_lattices_bitwise(precision):
    """Three instances with the perturbation operator in one batch, 41 steps (graph launches
    and eager ones): each equals the plain lattice run alone, bitwise."""
    ws = [inputs.double_droplet(n, n / 5.0, 1.0, 1.3, seed=40 + n, steps=0) for n in (40, 57, 64)]
    ps = [lbm3.make_params(w.nx, w.ny, SIG, TAU, precision=precision, forcing=PT) for w in ws]
    b = lbm3.lbm3_batch_create(ps)
    try:
        for i, w in enumerate(ws):
            lbm3.lbm3_batch_init_fields(b, i, w.rho)
        lbm3.lbm3_batch_step(b, 41)
        for i, w in enumerate(ws):
            _, rho = lbm3.lbm3_batch_observables(b, i, w.nx, w.ny, want_rho=True)
            L = lbm3.Lattice(w.nx, w.ny, SIG, TAU, precision=precision, forcing=PT).init(w.rho).step(41)
            ref = L.densities()
            L.close()
            assert np.array_equal(rho, ref), i
    finally:
        lbm3.lbm3_batch_destroy(b)


def test_refusals():
    """The adjoint covers the paper's forcing only; a batch takes one forcing."""
    L = lbm3.Lattice(16, 16, SIG, TAU, forcing=PT).init(inputs.random_mixture(16, 16, 1))
    try:
        with pytest.raises(lbm3.Lbm3Error) as e:
            lbm3.lbm3_adjoint_record(L.h, 2, 1)
        assert e.value.code == lbm3.LBM3_EUNSUPPORTED
    finally:
        L.close()
    with pytest.raises(lbm3.Lbm3Error) as e:
        lbm3.lbm3_batch_create([lbm3.make_params(16, 16), lbm3.make_params(16, 16, forcing=PT)])
    assert e.value.code == lbm3.LBM3_EINVAL


TABLE2 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table2_umax.json")))


def test_table2_perturbation_row():
    """The set-up of Table 2 (160^2 compound droplet, R_g = 2 R_r, all tensions 0.01, nu = 0.1)
    with the perturbation operator: after 80000 steps the maximum spurious velocity equals
    the table's second row to its printed digits (3.15, 3.28, 3.27, 3.29 x 1e-5 for
    R_r = 15..30), the Laplace jump stays within Table 1's band, and at R_r = 20 Guo forcing
    gives the smaller spurious velocity, as the paper reports."""
    got = []
    for Rr, want in zip(TABLE2["R_r"], TABLE2["u_max_x1e5"]["perturbation"]):
        w = inputs.compound_droplet(160, float(Rr), 2.0 * Rr, 0.01, 0.01, sigma_rb=0.01, tau=(0.8, 0.8, 0.8))
        L = lbm3.Lattice(160, 160, w.sigma, w.tau, forcing=PT).init(w.rho)
        obs, rho, _ = L.step(80000).observables(want_rho=True)
        L.close()
        lap = compound_laplace(rho, 80.0, 80.0, 0.01, 0.01)
        print(f"R_r={Rr}: u_max={obs['u_max'] * 1e5:.4f}e-5 (printed {want}e-5) eps={lap['eps'] * 100:.2f}%")
        got.append(obs["u_max"])
        assert abs(obs["u_max"] * 1e5 - want) <= 0.006
        assert lap["eps"] < 0.015
    w = inputs.compound_droplet(160, 20.0, 40.0, 0.01, 0.01, sigma_rb=0.01, tau=(0.8, 0.8, 0.8))
    L = lbm3.Lattice(160, 160, w.sigma, w.tau).init(w.rho)
    guo = L.step(80000).observables()[0]["u_max"]
    L.close()
    print(f"R_r=20 Guo forcing: u_max={guo * 1e5:.4f}e-5")
    assert guo < 0.5 * got[1]
