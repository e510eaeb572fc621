"""The hand-written adjoint through the C ABI, against central finite differences of the
FP64 oracle (h = 1e-6): gradients of L = sum_x (rho_1(x, T) - rho*(x))^2 with respect to
the three interfacial tensions and the initial densities."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1808_08555_amd import inputs, lbm3

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
SIGMA = (0.006, 0.010, 0.012)  # a strict Neumann triangle: |X_kl| < 1 for every pair


def sharp_janus(nx, ny, R):
    """A disk of fluids 0 | 1 (split at the centre column) in fluid 2, as the 256^2 case.
    Pure fluids have exactly zero colour gradients (guarded, no derivative), so the loss
    is smooth in the directions the tests perturb: tensions, and each node's own fluid."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    xc, yc = nx / 2.0, ny / 2.0
    inside = (x - xc) ** 2 + (y - yc) ** 2 <= R * R
    lab = np.full((ny, nx), 2)
    lab[inside & (x < xc)] = 0
    lab[inside & (x >= xc)] = 1
    return inputs.rho_from_labels(lab), lab


def gpu_gradient(rho0, target, sigma, tau, steps, every, tile=None):
    """tile = (threads, rows) sets a row-march shape, which keeps the forward's one-step
    launches and the reverse steps on the march."""
    ny, nx = rho0.shape[1:]
    L = lbm3.Lattice(nx, ny, sigma, tau).init(rho0)
    if tile is not None:
        lbm3.lbm3_set_tile(L.h, *tile)
    lbm3.lbm3_adjoint_record(L.h, steps, every)
    rho_T = L.densities()
    g = 2.0 * (rho_T[0] - target)
    ds, dr = lbm3.lbm3_adjoint(L.h, g, nx, ny)
    loss = float(((rho_T[0] - target) ** 2).sum())
    obs = L.observables()[0]
    L.close()
    assert obs["step"] == steps
    return loss, ds, dr


def oracle_loss(rho0, target, sigma, tau, steps):
    ny, nx = rho0.shape[1:]
    p = oracle.Params(nx, ny, tuple(sigma), tuple(tau))
    f = oracle.run(p, oracle.init(p, rho0), steps)
    return float(((f[0].sum(axis=0) - target) ** 2).sum())


@pytest.mark.parametrize("steps,every", [(1, 1), (4, 2), (12, 4), (30, 10)])
def test_adjoint_matches_oracle_finite_differences(steps, every):
    nx, ny, h = 24, 20, 1e-6
    tau = (0.7, 0.8, 0.9)
    rho0, lab = sharp_janus(nx, ny, 6.0)
    target = inputs.loss_target(rho0[0], seed=5550)
    loss, ds, dr = gpu_gradient(rho0, target, SIGMA, tau, steps, every)
    assert abs(loss / oracle_loss(rho0, target, SIGMA, tau, steps) - 1) < 1e-12
    for q in range(3):
        sp, sm = list(SIGMA), list(SIGMA)
        sp[q] += h
        sm[q] -= h
        fd = (oracle_loss(rho0, target, sp, tau, steps) - oracle_loss(rho0, target, sm, tau, steps)) / (2 * h)
        print(f"T={steps} dL/dsigma[{q}] adjoint {ds[q]:.10e} fd {fd:.10e}")
        assert abs(ds[q] - fd) <= 1e-5 * max(1e-3, abs(fd))
    rng = np.random.default_rng(steps)
    nodes = [(10, 7), (10, 12), (9, 14), (16, 10)] + [tuple(rng.integers(0, (ny, nx))) for _ in range(3)]
    for (y, x) in nodes:
        k = int(lab[y, x])
        rp, rm = rho0.copy(), rho0.copy()
        rp[k, y, x] += h
        rm[k, y, x] -= h
        fd = (oracle_loss(rp, target, SIGMA, tau, steps) - oracle_loss(rm, target, SIGMA, tau, steps)) / (2 * h)
        print(f"T={steps} dL/drho0[{k},{y},{x}] adjoint {dr[k, y, x]:.10e} fd {fd:.10e}")
        assert abs(dr[k, y, x] - fd) <= 1e-5 * max(1e-3, abs(fd))


def test_adjoint_wide_lattice_many_tiles_against_oracle_finite_differences():
    """1030 x 12 (wider than 1024, not a multiple of 16) with a march shape set, so the
    reverse sweep's row-marching pass runs as several strips and row segments.  Wavy vertical bands of the three fluids put
    interfaces across every strip and segment boundary and across the periodic seam; the
    probed nodes sit on strip boundaries (every 206 columns) and on the seam.  The loss here
    is about 400, so central differences at h = 1e-6 would carry about 4e-8 of rounding
    noise (eps L / h); h = 1e-4 keeps both that and the O(h^2) error near 1e-10."""
    nx, ny, h, steps, every = 1030, 12, 1e-4, 12, 4
    tau = (0.7, 0.8, 0.9)
    y, x = np.mgrid[0:ny, 0:nx]
    lab = ((x + np.round(2.5 * np.sin(2 * np.pi * y / ny)).astype(int)) // 7) % 3
    rho0 = inputs.rho_from_labels(lab)
    target = inputs.loss_target(rho0[0], seed=1030)
    loss, ds, dr = gpu_gradient(rho0, target, SIGMA, tau, steps, every, tile=(256, 0))
    assert abs(loss / oracle_loss(rho0, target, SIGMA, tau, steps) - 1) < 1e-12
    _, ds_b, dr_b = gpu_gradient(rho0, target, SIGMA, tau, steps, every)  # the fused block step
    assert np.allclose(ds_b, ds, rtol=1e-10, atol=0) and np.allclose(dr_b, dr, rtol=1e-9, atol=1e-12)
    for q in range(3):
        sp, sm = list(SIGMA), list(SIGMA)
        sp[q] += h
        sm[q] -= h
        fd = (oracle_loss(rho0, target, sp, tau, steps) - oracle_loss(rho0, target, sm, tau, steps)) / (2 * h)
        print(f"dL/dsigma[{q}] adjoint {ds[q]:.10e} fd {fd:.10e}")
        assert abs(ds[q] - fd) <= 1e-5 * max(1e-3, abs(fd))
    nodes = [(0, 0), (5, 1029), (11, 205), (3, 206), (7, 411), (8, 412), (2, 618), (10, 824), (6, 515)]
    for (yy, xx) in nodes:
        k = int(lab[yy, xx])
        rp, rm = rho0.copy(), rho0.copy()
        rp[k, yy, xx] += h
        rm[k, yy, xx] -= h
        fd = (oracle_loss(rp, target, SIGMA, tau, steps) - oracle_loss(rm, target, SIGMA, tau, steps)) / (2 * h)
        print(f"dL/drho0[{k},{yy},{xx}] adjoint {dr[k, yy, xx]:.10e} fd {fd:.10e}")
        assert abs(dr[k, yy, xx] - fd) <= 1e-5 * max(1e-3, abs(fd))


@pytest.mark.parametrize("shape", [(1, 1), (3, 2), (2, 7), (1, 40), (70, 1), (29, 13), (37, 29)])
def test_adjoint_fused_block_equals_march_on_tiny_and_ragged_lattices(shape):
    """The fused block reverse step (and the block recompute) against the row march (a march
    shape set) on lattices narrower than the halo, one-block lattices and ragged blocks:
    random three-fluid mixtures with near-zero entries, 6 steps with a checkpoint every 2.
    Each node's arithmetic is the same on both paths; only the dL/dsigma partial sums add in
    another order, and the back end may contract multiply-adds differently per kernel."""
    nx, ny = shape
    rho0 = inputs.random_mixture(nx, ny, 11, tiny_fraction=0.05)
    tau = (0.7, 0.8, 0.9)
    target = inputs.loss_target(rho0[0], seed=77)
    loss, ds, dr = gpu_gradient(rho0, target, SIGMA, tau, 6, 2)
    loss_m, ds_m, dr_m = gpu_gradient(rho0, target, SIGMA, tau, 6, 2, tile=(64, 0))
    assert loss == loss_m
    assert abs(loss / oracle_loss(rho0, target, SIGMA, tau, 6) - 1) < 1e-12
    assert np.isfinite(ds).all() and np.isfinite(dr).all()
    assert np.allclose(ds, ds_m, rtol=1e-9, atol=1e-12 * np.abs(ds_m).max()), (ds, ds_m)
    assert np.abs(dr - dr_m).max() <= 1e-11 * max(np.abs(dr_m).max(), 1e-300)


@pytest.mark.parametrize("n", [384, 1024])
def test_adjoint_block_pass_against_march_and_gpu_finite_differences(n):
    """Lattices past the fused reverse step's 2^17 nodes, up to the block pass's 2^20
    (384^2, 1024^2): the reverse steps run k_adj_local and the two-dimensional block pass.
    Janus droplet of radius 3n/16, 6 steps with a checkpoint every 2.  The gradients equal
    those of the row march (a march shape set) to summation order, and dL/dsigma matches
    central differences of the FP64 forward loss as in the 2048^2 case."""
    steps, h = 6, 1e-6
    w = inputs.janus_halves(n, 3 * n / 16, SIGMA, (0.8, 0.8, 0.8), steps)
    target = inputs.loss_target(w.rho[0], seed=5551)
    loss, ds, dr = gpu_gradient(w.rho, target, SIGMA, w.tau, steps, 2)
    loss_m, ds_m, dr_m = gpu_gradient(w.rho, target, SIGMA, w.tau, steps, 2, tile=(256, 0))
    assert loss == loss_m
    assert np.allclose(ds, ds_m, rtol=1e-10, atol=0), (ds, ds_m)
    scale = np.abs(dr_m).max()
    assert np.abs(dr - dr_m).max() <= 1e-12 * scale

    def L_at(sig):
        M = lbm3.Lattice(n, n, sig, w.tau).init(w.rho).step(steps)
        v = float(((M.densities()[0] - target) ** 2).sum())
        M.close()
        return v

    noise = 4 * 2.2e-16 * loss / h
    for q in range(3):
        sp, sm = list(SIGMA), list(SIGMA)
        sp[q] += h
        sm[q] -= h
        fd = (L_at(sp) - L_at(sm)) / (2 * h)
        print(f"n={n} dL/dsigma[{q}] adjoint {ds[q]:.10e} fd {fd:.10e} (noise {noise:.1e})")
        assert abs(ds[q] - fd) <= 1e-5 * abs(fd) + noise


def test_adjoint_above_the_overlap_size_against_gpu_finite_differences():
    """2048^2 (2^22 nodes: the sweep runs its segments one after the other in one slot,
    where smaller lattices overlap the next segment's recompute with the reverse steps),
    Janus droplet, 6 steps with a checkpoint every 2: dL/dsigma against central differences
    of the FP64 forward loss (the forward matches the oracle elsewhere), h = 1e-6, within
    1e-5 relative plus the differences' rounding noise (4 eps L / h)."""
    n, steps, h = 2048, 6, 1e-6
    w = inputs.janus_halves(n, 320.0, SIGMA, (0.8, 0.8, 0.8), steps)
    target = inputs.loss_target(w.rho[0], seed=5550)
    loss, ds, _ = gpu_gradient(w.rho, target, SIGMA, w.tau, steps, 2)

    def L_at(sig):
        M = lbm3.Lattice(n, n, sig, w.tau).init(w.rho).step(steps)
        v = float(((M.densities()[0] - target) ** 2).sum())
        M.close()
        return v

    noise = 4 * 2.2e-16 * loss / h
    for q in range(3):
        sp, sm = list(SIGMA), list(SIGMA)
        sp[q] += h
        sm[q] -= h
        fd = (L_at(sp) - L_at(sm)) / (2 * h)
        print(f"dL/dsigma[{q}] adjoint {ds[q]:.10e} fd {fd:.10e} (noise {noise:.1e})")
        assert abs(ds[q] - fd) <= 1e-5 * abs(fd) + noise


def test_adjoint_taylor_remainder_is_second_order():
    """With the GPU forward alone: L(rho0 + e d) - L(rho0) - e <grad, d> shrinks as e^2
    (d perturbs each node's own fluid)."""
    nx, ny = 32, 28
    rho0, lab = sharp_janus(nx, ny, 8.0)
    target = inputs.loss_target(rho0[0], seed=7)
    loss, ds, dr = gpu_gradient(rho0, target, SIGMA, (0.8, 0.8, 0.8), 20, 5)
    d = np.zeros_like(rho0)
    u = np.random.default_rng(3).uniform(-1, 1, lab.shape) * 0.01
    for k in range(3):
        d[k][lab == k] = u[lab == k]

    def L_at(r):
        M = lbm3.Lattice(nx, ny, SIGMA, (0.8, 0.8, 0.8)).init(r).step(20)
        v = float(((M.densities()[0] - target) ** 2).sum())
        M.close()
        return v

    lin = float((dr * d).sum())
    rem = [abs(L_at(rho0 + e * d) - loss - e * lin) for e in (1e-2, 5e-3, 2.5e-3)]
    print("Taylor remainders:", rem, "first-order term", 1e-2 * lin)
    assert rem[1] / rem[0] < 0.3 and rem[2] / rem[1] < 0.3  # ~1/4 for a second-order remainder


def test_adjoint_janus_256_5000_steps_against_stored_finite_differences():
    """The 256^2 Janus droplet of two half-disks (R = 40), 5000 steps with a checkpoint every
    100: the adjoint gradient against central differences of the oracle stored by
    tests/golden/make_adjoint_fd.py."""
    path = os.path.join(HERE, "golden", "janus256_fd.json")
    ref = json.load(open(path))
    w = inputs.janus_halves(256, 40.0, SIGMA, (0.8, 0.8, 0.8), ref["steps"])
    target = inputs.loss_target(w.rho[0], seed=5550)
    loss, ds, dr = gpu_gradient(w.rho, target, SIGMA, w.tau, ref["steps"], 100)
    print("loss gpu", loss, "oracle", ref["loss"])
    assert abs(loss / ref["loss"] - 1) < 1e-9
    for q in range(3):
        fd = ref["dL_dsigma"][q]
        print(f"dL/dsigma[{q}] adjoint {ds[q]:.10e} fd {fd:.10e}")
        assert abs(ds[q] - fd) <= 1e-4 * abs(fd)
    for k, y, x, fd in ref["dL_drho0"]:
        print(f"dL/drho0[{k},{y},{x}] adjoint {dr[k, y, x]:.10e} fd {fd:.10e}")
        assert abs(dr[k, y, x] - fd) <= 1e-4 * max(abs(fd), 1e-3)


def test_adjoint_errors():
    L = lbm3.Lattice(8, 8)
    rho = inputs.random_mixture(8, 8, 1, tiny_fraction=0.0)
    with pytest.raises(lbm3.Lbm3Error):
        lbm3.lbm3_adjoint(L.h, np.zeros((8, 8)), 8, 8)  # no recording yet
    L.init(rho).step(1)
    with pytest.raises(lbm3.Lbm3Error) as e:
        lbm3.lbm3_adjoint_record(L.h, 4, 2)  # not at step 0
    assert e.value.code == lbm3.LBM3_ESTATE
    L.init(rho)
    with pytest.raises(lbm3.Lbm3Error):
        lbm3.lbm3_adjoint_record(L.h, 5, 2)  # not a multiple
    L.close()
    F = lbm3.Lattice(8, 8, precision="fp32").init(rho)
    with pytest.raises(lbm3.Lbm3Error) as e:
        lbm3.lbm3_adjoint_record(F.h, 2, 1)
    assert e.value.code == lbm3.LBM3_EUNSUPPORTED
    F.close()
