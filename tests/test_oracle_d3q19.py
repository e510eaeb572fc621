"""The D3Q19 oracle (the three-dimensional form of the ternary step) pinned to the
two-dimensional oracle and to symmetries.  D3Q19's weights summed over the links that share
an in-plane direction are D2Q9's, and every part of the step is linear in those sums or
depends only on in-plane components when the fields are uniform along one axis.  So a
lattice uniform along z (or x, or y) must evolve, population sums over the out-of-plane
link component, exactly as the pinned two-dimensional oracle.  Swapping two axes of the
input must swap them in the output.  Planted mistakes in a copy of the source are caught."""
import os

import numpy as np
import pytest

import oracle
from oracle import d3q19
from paper_1808_08555_amd import inputs

SIG, TAU = (0.011, 0.013, 0.017), (0.7, 1.0, 1.3)
EX2 = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY2 = [0, 0, 1, 0, -1, 1, 1, -1, -1]
PLANES = {"z": (0, 1), "x": (1, 2), "y": (2, 0)}  # invariant axis -> in-plane axes (a, b); 0=x 1=y 2=z


def lift(rho2, axis, m):
    """rho2 [3, n_b, n_a] -> rho3 [3, nz, ny, nx], uniform along `axis` (length m)."""
    if axis == "z":
        return np.repeat(rho2[:, None, :, :], m, axis=1)
    if axis == "x":  # a = y, b = z: rho3[k, z, y, x] = rho2[k, z, y]
        return np.repeat(rho2[:, :, :, None], m, axis=3)
    # axis == "y": a = z, b = x: rho3[k, z, y, x] = rho2[k, x, z]
    return np.repeat(np.transpose(rho2, (0, 2, 1))[:, :, None, :], m, axis=2)


def project(f3, axis):
    """f3 [3, 19, nz, ny, nx] -> [3, 9, n_b, n_a]: populations summed over the links with
    the same in-plane components, one slice along the uniform axis."""
    e, _ = d3q19.lattice()
    a, b = PLANES[axis]
    if axis == "z":
        sl = f3[:, :, 0, :, :]
    elif axis == "x":
        sl = f3[:, :, :, :, 0]
    else:
        sl = np.transpose(f3[:, :, :, 0, :], (0, 1, 3, 2))
    out = np.zeros((3, 9) + sl.shape[2:])
    for q in range(9):
        for i in range(19):
            if e[i, a] == EX2[q] and e[i, b] == EY2[q]:
                out[:, q] += sl[:, i]
    return out


def run3(rho3, steps, sigma=SIG, tau=TAU, law="paper"):
    nz, ny, nx = rho3.shape[1:]
    p = oracle.Params(nx, ny, sigma, tau, beta_law=law)
    return d3q19.run(p, nz, d3q19.init(p, nz, rho3), steps)


@pytest.mark.parametrize("axis", ["z", "x", "y"])
@pytest.mark.parametrize("m", [1, 3])
def test_uniform_along_an_axis_reduces_to_the_2d_oracle(axis, m):
    na, nb, steps = 11, 9, 6
    rho2 = inputs.random_mixture(na, nb, 7, tiny_fraction=0.05)
    f3 = run3(lift(rho2, axis, m), steps)
    p2 = oracle.Params(na, nb, SIG, TAU)
    f2 = oracle.run(p2, oracle.init(p2, rho2), steps)
    err = np.abs(project(f3, axis) - f2).max()
    print(axis, m, err)
    assert err < 1e-13


def test_uniform_along_z_with_a_comparison_law():
    rho2 = inputs.random_mixture(10, 8, 3, tiny_fraction=0.0)
    f3 = run3(lift(rho2, "z", 2), 4, law="leclaire")
    p2 = oracle.Params(10, 8, SIG, TAU, beta_law="leclaire")
    assert np.abs(project(f3, "z") - oracle.run(p2, oracle.init(p2, rho2), 4)).max() < 1e-13


def _random3(n=(7, 6, 5), seed=2):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.05, 1.05, (3,) + n)


def test_conservation_in_three_dimensions():
    rho3 = _random3()
    nz, ny, nx = rho3.shape[1:]
    p = oracle.Params(nx, ny, SIG, TAU)
    f0 = d3q19.init(p, nz, rho3)
    f1 = d3q19.run(p, nz, f0, 3)
    e, _ = d3q19.lattice()
    assert np.abs(f1.sum(axis=(1, 2, 3, 4)) / f0.sum(axis=(1, 2, 3, 4)) - 1).max() < 1e-14
    mom = [(f1.sum(0) * e[:, a][:, None, None, None]).sum() for a in range(3)]
    assert np.abs(mom).max() < 1e-13  # at rest initially; no net force on a periodic lattice


@pytest.mark.parametrize("swap", [(0, 1), (1, 2), (0, 2)])
def test_swapping_two_axes_commutes_with_the_step(swap):
    n = 6
    rho3 = _random3((n, n, n), seed=5)
    e, _ = d3q19.lattice()
    arr_axis = {0: 3, 1: 2, 2: 1}  # lattice axis -> array axis of rho [3, z, y, x]
    A, B = arr_axis[swap[0]], arr_axis[swap[1]]
    rho_s = np.swapaxes(rho3, A, B).copy()
    perm = []
    for i in range(19):
        v = e[i].copy()
        v[list(swap)] = v[list(swap[::-1])]
        perm.append(int(np.where((e == v).all(axis=1))[0][0]))
    f = run3(rho3, 2)
    fs = run3(rho_s, 2)
    # f'_{perm[i]} (swapped position) = f_i (position)
    want = np.swapaxes(f, A + 1, B + 1)[:, np.argsort(perm)]
    assert np.abs(fs - want).max() < 1e-14


MUTANTS = {
    "edge_weight": ("(i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0)", "(i <= 6 ? 1.0 / 18.0 : 1.0 / 18.0)"),
    "gradient_factor": ("d[a * g->N + j] = 3.0 * s[a];", "d[a * g->N + j] = s[a];"),
    "edge_link_z_sign": ("{1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},",
                         "{1, 0, 1},   {-1, 0, -1}, {1, 0, 1}, {-1, 0, -1},"),
    "stress_projector": ("((u == v ? 1.0 : 0.0) - n[u] * n[v]);", "((u == v ? 1.0 : 0.0) - n[u] * n[u]);"),
    "force_transposed": ("F[b * N + j] += d[a * N + j];", "F[b * N + j] += d[b * N + j];"),
    "no_half_force": ("u[a] = (m[a] + 0.5 * Fv[a]) / r;", "u[a] = m[a] / r;"),
    "recolour_direction": ("(n[0] * E3[i][0] + n[1] * E3[i][1] + n[2] * E3[i][2])",
                           "(n[0] * E3[i][0] + n[1] * E3[i][2] + n[2] * E3[i][1])"),
}


def _pins():
    yield lambda: test_uniform_along_an_axis_reduces_to_the_2d_oracle("z", 1)
    yield lambda: test_uniform_along_an_axis_reduces_to_the_2d_oracle("x", 3)
    yield lambda: test_uniform_along_an_axis_reduces_to_the_2d_oracle("y", 3)
    yield test_conservation_in_three_dimensions
    for s in [(0, 1), (1, 2), (0, 2)]:
        yield lambda s=s: test_swapping_two_axes_commutes_with_the_step(s)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = d3q19.source_text()
    assert src.count(old) == 1, f"pattern for {name} must occur exactly once"
    so = d3q19.compile_source(src.replace(old, new), os.path.join(tmp_path, f"mut_{name}.so"))
    caught = None
    with d3q19.use_library(so):
        for pin in _pins():
            try:
                pin()
            except AssertionError as e:
                caught = e
                break
    assert caught is not None, f"no pin catches the planted mistake {name}"
