"""The three-dimensional oracle (the ternary step on D3Q19 and D3Q27) pinned to the
two-dimensional oracle, to closed forms and to symmetries.  On either lattice the weights
summed over the links that share an in-plane direction are D2Q9's (D3Q19: 1/3 + 2/18,
1/18 + 2/36, 1/36; D3Q27: 8/27 + 4/27, 2/27 + 2/54, 1/54 + 2/216), and every part of the
step is linear in those sums or depends only on in-plane components when the fields are
uniform along one axis.  So a lattice uniform along z (or x, or y) must evolve, population
sums over the out-of-plane link component, exactly as the pinned two-dimensional oracle.
The weights must have the moments of an isotropic lattice with c_s^2 = 1/3.  Swapping two
axes of the input must swap them in the output.  Planted mistakes in a copy of the source
are caught."""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import d3
from paper_1808_08555_amd import inputs

SIG, TAU = (0.011, 0.013, 0.017), (0.7, 1.0, 1.3)
EX2 = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY2 = [0, 0, 1, 0, -1, 1, 1, -1, -1]
PLANES = {"z": (0, 1), "x": (1, 2), "y": (2, 0)}  # invariant axis -> in-plane axes (a, b); 0=x 1=y 2=z
QS = [19, 27]


def lift(rho2, axis, m):
    """rho2 [3, n_b, n_a] -> rho3 [3, nz, ny, nx], uniform along `axis` (length m)."""
    if axis == "z":
        return np.repeat(rho2[:, None, :, :], m, axis=1)
    if axis == "x":  # a = y, b = z: rho3[k, z, y, x] = rho2[k, z, y]
        return np.repeat(rho2[:, :, :, None], m, axis=3)
    # axis == "y": a = z, b = x: rho3[k, z, y, x] = rho2[k, x, z]
    return np.repeat(np.transpose(rho2, (0, 2, 1))[:, :, None, :], m, axis=2)


def project(f3, axis):
    """f3 [3, q, nz, ny, nx] -> [3, 9, n_b, n_a]: populations summed over the links with
    the same in-plane components, one slice along the uniform axis."""
    q3 = f3.shape[1]
    e, _ = d3.lattice(q3)
    a, b = PLANES[axis]
    if axis == "z":
        sl = f3[:, :, 0, :, :]
    elif axis == "x":
        sl = f3[:, :, :, :, 0]
    else:
        sl = np.transpose(f3[:, :, :, 0, :], (0, 1, 3, 2))
    out = np.zeros((3, 9) + sl.shape[2:])
    for q in range(9):
        for i in range(q3):
            if e[i, a] == EX2[q] and e[i, b] == EY2[q]:
                out[:, q] += sl[:, i]
    return out


def run3(rho3, steps, sigma=SIG, tau=TAU, law="paper", q=19):
    nz, ny, nx = rho3.shape[1:]
    p = oracle.Params(nx, ny, sigma, tau, beta_law=law)
    return d3.run(p, nz, d3.init(p, nz, rho3, q), steps)


@pytest.mark.parametrize("q", QS)
def test_lattice_moments(q):
    """sum w = 1, sum w e = 0, sum w e_a e_b = delta_ab / 3, odd moments zero and
    sum w e_a e_b e_c e_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 9; every link's opposite
    follows it; D3Q19 is the first 19 links of D3Q27."""
    e, w = d3.lattice(q)
    assert len(set(map(tuple, e))) == q and (w > 0).all()
    assert abs(w.sum() - 1) < 1e-15
    d = np.eye(3)
    for n in (1, 3, 5):
        for idx in itertools.product(range(3), repeat=n):
            assert abs((w * np.prod([e[:, a] for a in idx], axis=0)).sum()) < 1e-15
    for a, b in itertools.product(range(3), repeat=2):
        assert abs((w * e[:, a] * e[:, b]).sum() - d[a, b] / 3) < 1e-15
    for a, b, c, g in itertools.product(range(3), repeat=4):
        want = (d[a, b] * d[c, g] + d[a, c] * d[b, g] + d[a, g] * d[b, c]) / 9
        assert abs((w * e[:, a] * e[:, b] * e[:, c] * e[:, g]).sum() - want) < 1e-15
    assert (e[2::2] == -e[1::2]).all()
    if q == 27:
        assert (d3.lattice(19)[0] == e[:19]).all()
        assert (np.abs(e).sum(axis=1)[19:] == 3).all()


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("axis", ["z", "x", "y"])
@pytest.mark.parametrize("m", [1, 3])
def test_uniform_along_an_axis_reduces_to_the_2d_oracle(axis, m, q):
    na, nb, steps = 11, 9, 6
    rho2 = inputs.random_mixture(na, nb, 7, tiny_fraction=0.05)
    f3 = run3(lift(rho2, axis, m), steps, q=q)
    p2 = oracle.Params(na, nb, SIG, TAU)
    f2 = oracle.run(p2, oracle.init(p2, rho2), steps)
    err = np.abs(project(f3, axis) - f2).max()
    print(q, axis, m, err)
    assert err < 1e-13


@pytest.mark.parametrize("q", QS)
def test_uniform_along_z_with_a_comparison_law(q):
    rho2 = inputs.random_mixture(10, 8, 3, tiny_fraction=0.0)
    f3 = run3(lift(rho2, "z", 2), 4, law="leclaire", q=q)
    p2 = oracle.Params(10, 8, SIG, TAU, beta_law="leclaire")
    assert np.abs(project(f3, "z") - oracle.run(p2, oracle.init(p2, rho2), 4)).max() < 1e-13


def _random3(n=(7, 6, 5), seed=2):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.05, 1.05, (3,) + n)


@pytest.mark.parametrize("q", QS)
def test_conservation_in_three_dimensions(q):
    rho3 = _random3()
    nz, ny, nx = rho3.shape[1:]
    p = oracle.Params(nx, ny, SIG, TAU)
    f0 = d3.init(p, nz, rho3, q)
    f1 = d3.run(p, nz, f0, 3)
    e, _ = d3.lattice(q)
    assert np.abs(f1.sum(axis=(1, 2, 3, 4)) / f0.sum(axis=(1, 2, 3, 4)) - 1).max() < 1e-14
    mom = [(f1.sum(0) * e[:, a][:, None, None, None]).sum() for a in range(3)]
    assert np.abs(mom).max() < 1e-13  # at rest initially; no net force on a periodic lattice


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("swap", [(0, 1), (1, 2), (0, 2)])
def test_swapping_two_axes_commutes_with_the_step(swap, q):
    n = 6
    rho3 = _random3((n, n, n), seed=5)
    e, _ = d3.lattice(q)
    arr_axis = {0: 3, 1: 2, 2: 1}  # lattice axis -> array axis of rho [3, z, y, x]
    A, B = arr_axis[swap[0]], arr_axis[swap[1]]
    rho_s = np.swapaxes(rho3, A, B).copy()
    perm = []
    for i in range(q):
        v = e[i].copy()
        v[list(swap)] = v[list(swap[::-1])]
        perm.append(int(np.where((e == v).all(axis=1))[0][0]))
    f = run3(rho3, 2, q=q)
    fs = run3(rho_s, 2, q=q)
    # f'_{perm[i]} (swapped position) = f_i (position)
    want = np.swapaxes(f, A + 1, B + 1)[:, np.argsort(perm)]
    assert np.abs(fs - want).max() < 1e-14


def test_d3q27_differs_from_d3q19_off_the_plane():
    """The two lattices agree on fields uniform along an axis (both reduce to D2Q9) but not
    on a genuinely three-dimensional field: the corner links change the answer."""
    rho3 = _random3((6, 6, 6), seed=9)
    f19, f27 = run3(rho3, 2, q=19), run3(rho3, 2, q=27)
    r19, r27 = f19.sum(axis=1), f27.sum(axis=1)
    assert np.abs(r19 - r27).max() > 1e-6


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
    "d3q27_corner_weight": ("(i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0)", "(i <= 18 ? 1.0 / 54.0 : 1.0 / 108.0)"),
    "d3q27_rest_weight": ("i == 0 ? 8.0 / 27.0 :", "i == 0 ? 7.0 / 27.0 :"),
    "d3q27_corner_link": ("{1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}",
                          "{1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, 1}"),
    "d3q27_gradient_skips_corners": ("for (int i = 1; i < g->q; i += 2) {", "for (int i = 1; i < 19; i += 2) {"),
}


def _pins():
    for q in QS:
        yield lambda q=q: test_lattice_moments(q)
        yield lambda q=q: test_uniform_along_an_axis_reduces_to_the_2d_oracle("z", 1, q)
        yield lambda q=q: test_uniform_along_an_axis_reduces_to_the_2d_oracle("x", 3, q)
        yield lambda q=q: test_uniform_along_an_axis_reduces_to_the_2d_oracle("y", 3, q)
        yield lambda q=q: test_conservation_in_three_dimensions(q)
        for s in [(0, 1), (1, 2), (0, 2)]:
            yield lambda s=s, q=q: test_swapping_two_axes_commutes_with_the_step(s, q)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = d3.source_text()
    assert src.count(old) == 1, f"pattern for {name} must occur exactly once"
    so = d3.compile_source(src.replace(old, new), os.path.join(tmp_path, f"mut_{name}.so"))
    caught = None
    with d3.use_library(so):
        for pin in _pins():
            try:
                pin()
            except (AssertionError, IndexError, ValueError) as e:
                caught = e
                break
    assert caught is not None, f"no pin catches the planted mistake {name}"
