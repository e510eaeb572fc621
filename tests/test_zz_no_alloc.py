"""The allocation-free observables entry point (lbm3_observables_noalloc) through the C ABI:
its result equals lbm3_observables' bit for bit, on consecutive calls whose second one
covers a smaller lattice (the shared static scratch keeps the first call's contents), and a
launch plan larger than the scratch is refused before any device work."""
import numpy as np
import pytest

from paper_1808_08555_amd import inputs, lbm3

pytestmark = pytest.mark.gpu


def _same(a: dict, b: dict):
    assert a["step"] == b["step"]
    assert np.array_equal(a["mass"], b["mass"])
    assert np.array_equal(a["momentum"], b["momentum"])
    assert a["kinetic_energy"] == b["kinetic_energy"]
    assert a["u_max"] == b["u_max"]
    assert a["nonfinite"] == b["nonfinite"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_storage", "fp32"])
def test_noalloc_observables_equal_the_allocating_call(precision):
    big = inputs.double_droplet(301, 40.0, 1.0, 1.3, seed=3, steps=0)
    small = inputs.double_droplet(40, 8.0, 1.0, 1.3, seed=11, steps=0)
    Lb = lbm3.Lattice(big.nx, big.ny, big.sigma, big.tau, precision=precision).init(big.rho).step(31)
    Ls = lbm3.Lattice(small.nx, small.ny, small.sigma, small.tau, precision=precision).init(small.rho).step(17)
    try:
        # two calls in a row on the shared scratch, the second on the smaller lattice
        nb = lbm3.lbm3_observables_noalloc(Lb.h)
        ns = lbm3.lbm3_observables_noalloc(Ls.h)
        _same(nb, Lb.observables()[0])
        _same(ns, Ls.observables()[0])
        assert nb["step"] == 31 and ns["step"] == 17
        assert nb["mass"][2] > ns["mass"][2] > 0
        # and again after more steps, in the other order
        Lb.step(2)
        Ls.step(3)
        ns = lbm3.lbm3_observables_noalloc(Ls.h)
        nb = lbm3.lbm3_observables_noalloc(Lb.h)
        _same(ns, Ls.observables()[0])
        _same(nb, Lb.observables()[0])
    finally:
        Lb.close()
        Ls.close()


def test_noalloc_observables_refuse_a_plan_beyond_the_scratch():
    L = lbm3.Lattice(2048, 1024, precision="fp32")
    try:
        rho = np.zeros((3, 1024, 2048))
        rho[2] = 1.0
        L.init(rho)
        L.set_tile(64, 1)  # 36 strips x 1024 one-row segments: more than 32768 workgroups
        with pytest.raises(lbm3.Lbm3Error) as e:
            lbm3.lbm3_observables_noalloc(L.h)
        assert e.value.code == lbm3.LBM3_EINVAL and "32768" in str(e.value)
        L.set_tile(256, 0)
        o = lbm3.lbm3_observables_noalloc(L.h)
        assert o["mass"][2] == 2048 * 1024
    finally:
        L.close()
