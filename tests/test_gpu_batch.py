"""The batched form through the C ABI: parity with the plain step and the oracle, graph
replays, observables, the autotuner, and the morphology classes of the sweep."""
import numpy as np
import pytest

import oracle
from paper_1808_08555_amd import autotune, inputs, lbm3, morphology

pytestmark = pytest.mark.gpu


def _batch_state(b, i, w):
    obs, rho = lbm3.lbm3_batch_observables(b, i, w.nx, w.ny, want_rho=True)
    return obs, rho


def _mixed_workloads():
    """Five instances of different sizes (ragged, not multiples of anything) and parameters."""
    ws = [inputs.double_droplet(40, 8.0, 1.0, 1.3, seed=1, steps=0),
          inputs.compound_droplet(64, 10.0, 20.0, 0.01, 0.005, tau=(0.7, 0.9, 1.1)),
          inputs.single_droplet(37, 9.0),
          inputs.Workload("rand", 23, 19, (0.011, 0.013, 0.017), (0.7, 1.0, 1.3),
                          rho=inputs.random_mixture(23, 19, 3, tiny_fraction=0.05)),
          inputs.double_droplet(96, 15.0, 0.5, 1.7, seed=2, steps=0)]
    return ws


def _make_batch(ws, precision):
    ps = [lbm3.make_params(w.nx, w.ny, w.sigma, w.tau, w.rho0, w.beta0, precision) for w in ws]
    b = lbm3.lbm3_batch_create(ps)
    for i, w in enumerate(ws):
        lbm3.lbm3_batch_init_fields(b, i, w.rho)
    return b


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_storage"])
def test_batch_matches_plain_step_bitwise(precision):
    """57 steps (two graph launches of 20 steps and 17 eager launches): every instance's
    densities equal those of the plain lattice run alone, bitwise.  With FP32 storage this
    also checks the stochastic rounding: the second graph replay must round with the salts of
    steps 21-40, as the plain lattice does, not with those of the captured steps 1-20."""
    ws = _mixed_workloads()
    b = _make_batch(ws, precision)
    lbm3.lbm3_batch_step(b, 40)
    lbm3.lbm3_batch_step(b, 17)
    for i, w in enumerate(ws):
        obs, rho = _batch_state(b, i, w)
        L = lbm3.Lattice(w.nx, w.ny, w.sigma, w.tau, w.rho0, w.beta0, precision).init(w.rho).step(57)
        ref = L.densities()
        L.close()
        assert obs["step"] == 57
        assert np.array_equal(rho, ref), (i, w.name)
    lbm3.lbm3_batch_destroy(b)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_storage"])
@pytest.mark.parametrize("threads", [0, 64, 256])
def test_batch_two_step_pass_matches_plain_step_bitwise(precision, threads):
    """With two steps per launch (graph of two-step launches, then eager pairs and an odd last
    step), every instance equals the plain lattice stepped one step per launch, bitwise."""
    ws = _mixed_workloads()
    b = _make_batch(ws, precision)
    if threads:
        lbm3.lbm3_batch_set_tile(b, 0, threads, 0)
    lbm3.lbm3_batch_set_steps_per_launch(b, 2)
    steps, t2, rows2, wg2 = lbm3.lbm3_batch_get_pair_launch(b)
    assert steps == 2 and t2 > 0 and rows2 > 0 and wg2 > 0
    lbm3.lbm3_batch_step(b, 1)   # 27-population -> factored, one step
    lbm3.lbm3_batch_step(b, 40)  # two graph launches
    lbm3.lbm3_batch_step(b, 16)  # seven pairs and one single step
    for i, w in enumerate(ws):
        obs, rho = _batch_state(b, i, w)
        L = lbm3.Lattice(w.nx, w.ny, w.sigma, w.tau, w.rho0, w.beta0, precision).init(w.rho)
        L.set_steps_per_launch(1).step(57)
        ref = L.densities()
        L.close()
        assert obs["step"] == 57
        assert np.array_equal(rho, ref), (i, w.name)
    lbm3.lbm3_batch_destroy(b)


def test_batch_matches_oracle_fp64():
    ws = _mixed_workloads()
    b = _make_batch(ws, "fp64")
    lbm3.lbm3_batch_step(b, 25)
    for i, w in enumerate(ws):
        _, rho = _batch_state(b, i, w)
        p = oracle.Params(w.nx, w.ny, w.sigma, w.tau, w.rho0, w.beta0)
        ref = oracle.density(oracle.run(p, oracle.init(p, w.rho), 25))
        assert np.abs(rho - ref).max() <= 1e-11, (i, w.name)
    lbm3.lbm3_batch_destroy(b)


def test_graph_replays_with_eager_work_between():
    """Graph replays interleaved with eager steps and host synchronisation give the same
    state as an all-eager run (steps in chunks below the graph length)."""
    ws = _mixed_workloads()
    a = _make_batch(ws, "fp64")
    c = _make_batch(ws, "fp64")
    for chunk in (20, 3, 40, 1, 20):
        lbm3.lbm3_batch_step(a, chunk)
        _batch_state(a, 0, ws[0])  # synchronising host work between replays
    for _ in range(84):
        lbm3.lbm3_batch_step(c, 1)
    for i, w in enumerate(ws):
        assert np.array_equal(_batch_state(a, i, w)[1], _batch_state(c, i, w)[1]), i
    lbm3.lbm3_batch_destroy(a)
    lbm3.lbm3_batch_destroy(c)


def test_batch_tile_shapes_bitwise():
    ws = _mixed_workloads()
    ref = None
    for t, r in [(64, 0), (128, 16), (256, 0), (512, 7)]:
        b = _make_batch(ws, "fp64")
        lbm3.lbm3_batch_set_tile(b, 0, t, r)
        lbm3.lbm3_batch_step(b, 30)
        got = [_batch_state(b, i, w)[1] for i, w in enumerate(ws)]
        lbm3.lbm3_batch_destroy(b)
        if ref is None:
            ref = got
        else:
            for i in range(len(ws)):
                assert np.array_equal(got[i], ref[i]), (t, r, i)


def test_batch_errors():
    ws = _mixed_workloads()[:2]
    ps = [lbm3.make_params(w.nx, w.ny, w.sigma, w.tau) for w in ws]
    b = lbm3.lbm3_batch_create(ps)
    with pytest.raises(lbm3.Lbm3Error) as e:
        lbm3.lbm3_batch_step(b, 1)
    assert e.value.code == lbm3.LBM3_ESTATE
    with pytest.raises(lbm3.Lbm3Error):
        lbm3.lbm3_batch_init_fields(b, 5, ws[0].rho)
    with pytest.raises(lbm3.Lbm3Error):
        lbm3.lbm3_batch_set_tile(b, 40, 100, 0)
    lbm3.lbm3_batch_destroy(b)
    mixed = [lbm3.make_params(8, 8, precision="fp64"), lbm3.make_params(8, 8, precision="fp32")]
    with pytest.raises(lbm3.Lbm3Error):
        lbm3.lbm3_batch_create(mixed)


def test_autotuner_choice_is_applied_and_cached(tmp_path, monkeypatch):
    monkeypatch.setenv("LBM3_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    t, r = autotune.tune_lattice(256, 256, "fp32", steps=5)
    assert t in autotune.THREADS and r in autotune.ROWS
    assert autotune.tune_lattice(256, 256, "fp32") == (t, r)  # served from the cache
    ws = _mixed_workloads()
    b = _make_batch(ws, "fp32")
    threads, rows = autotune.tune_batch(b, [w.nx for w in ws], "fp32", steps=4)
    assert threads in autotune.THREADS
    lbm3.lbm3_batch_step(b, 5)
    _batch_state(b, 0, ws[0])
    lbm3.lbm3_batch_destroy(b)


def test_autotuner_times_a_batch_on_its_own_stream():
    """A batch created without a stream orders its work on a stream of its own; the tuner's
    timing must still cover that work.  64 instances (6.3 M nodes) in FP32 move at least
    64 B per node and step, so a timing that implied more than the 8 TB/s HBM peak would
    have missed the kernels (launch overhead alone is a few microseconds per step)."""
    import torch
    ws = inputs.morphology_batch()
    b = _make_batch(ws, "fp32")
    try:
        nodes = sum(w.nx * w.ny for w in ws)
        ms = autotune._time(torch, lambda n: lbm3.lbm3_batch_step(b, n), 20)
        floor_ms = nodes * 64 / 8e12 * 1e3
        print(f"batch timing {ms:.4f} ms/step, HBM floor {floor_ms:.4f} ms/step")
        assert ms >= floor_ms
    finally:
        lbm3.lbm3_batch_destroy(b)


def _contact(c, a, b, lo=0.2):
    return int(((c[a] > lo) & (c[b] > lo)).sum())


def test_morphology_sweep_classes():
    """Sec. 4.1 morphologies on a subset of the 8 x 8 sweep (side 128, FP32, 20000 steps):
    where fluid 0 should engulf fluid 1 the matrix loses contact with fluid 1; where the
    droplets should stay separate they lose contact with each other; partial engulfing
    keeps all three contacts."""
    cases = {morphology.ENGULF_1_BY_0: (0.25, 0.25), morphology.SEPARATE: (2.0, 0.5),
             morphology.PARTIAL: (1.0, 1.0), morphology.ENGULF_0_BY_1: (0.25, 2.0)}
    ws = []
    for kind, (r12, r13) in cases.items():
        assert morphology.classify(r12 * 0.01, r13 * 0.01, 0.01) == kind
        side = 128
        R = side / 6.0
        c0 = side / 2.0
        disks = [(0, c0 - R, c0, R), (1, c0 + R, c0, R)]
        rho = inputs.rho_from_labels(inputs.label_disks(side, side, disks))
        ws.append(inputs.Workload(kind, side, side, (r12 * 0.01, r13 * 0.01, 0.01), rho=rho))
    b = _make_batch(ws, "fp32")
    lbm3.lbm3_batch_step(b, 20000)
    for i, (kind, w) in enumerate(zip(cases, ws)):
        _, rho = _batch_state(b, i, w)
        c = rho / rho.sum(0)
        rg, rb, gb = _contact(c, 0, 1), _contact(c, 0, 2), _contact(c, 1, 2)
        print(kind, "contacts rg/rb/gb:", rg, rb, gb)
        if kind == morphology.ENGULF_1_BY_0:
            assert gb <= 0.02 * rb and rg > 0
        elif kind == morphology.ENGULF_0_BY_1:
            assert rb <= 0.02 * gb and rg > 0
        elif kind == morphology.SEPARATE:
            assert rg <= 0.05 * min(rb, gb)
        else:
            assert rg > 0 and rb > 0 and gb > 0
    lbm3.lbm3_batch_destroy(b)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_reinitialised_instance_in_a_stepped_batch(precision):
    """Re-initialising one instance after the batch has stepped leaves it in the 27-population
    format next to factored ones; the next step runs both kinds (each launch skipping the
    other format) and every instance still equals its plain run bitwise."""
    ws = _mixed_workloads()
    b = _make_batch(ws, precision)
    lbm3.lbm3_batch_step(b, 30)
    fresh = inputs.single_droplet(37, 7.0)
    assert (fresh.nx, fresh.ny) == (ws[2].nx, ws[2].ny)
    lbm3.lbm3_batch_init_fields(b, 2, fresh.rho)
    lbm3.lbm3_batch_step(b, 25)
    for i, w in enumerate(ws):
        _, rho = _batch_state(b, i, w)
        if i == 2:
            L = lbm3.Lattice(w.nx, w.ny, w.sigma, w.tau, w.rho0, w.beta0, precision).init(fresh.rho).step(25)
        else:
            L = lbm3.Lattice(w.nx, w.ny, w.sigma, w.tau, w.rho0, w.beta0, precision).init(w.rho).step(55)
        ref = L.densities()
        L.close()
        assert np.array_equal(rho, ref), (i, w.name)
    lbm3.lbm3_batch_destroy(b)


def test_morphology_batch_in_the_benchmark_plan_matches_plain_bitwise(monkeypatch, tmp_path):
    """The batched form exactly as the benchmark runs it: the 64-instance morphology sweep
    (sides 128-512, FP32) with the autotuner's plan (the two-step launch where it wins),
    200 steps (ten replays of the captured graph): every instance's densities equal the
    same lattice stepped alone, bit for bit.  The tuning goes to a cache of the test's own."""
    monkeypatch.setenv("LBM3_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    ws = inputs.morphology_batch()
    b = _make_batch(ws, "fp32")
    try:
        autotune.tune_batch(b, [w.nx for w in ws], "fp32", steps=20)
        plan = lbm3.lbm3_batch_get_pair_launch(b)
        print("benchmark plan (steps per launch, threads, rows, workgroups):", plan)
        for i, w in enumerate(ws):  # tuning stepped the batch: start again from the inputs
            lbm3.lbm3_batch_init_fields(b, i, w.rho)
        lbm3.lbm3_batch_step(b, 200)
        for i, w in enumerate(ws):
            _, rho = _batch_state(b, i, w)
            L = lbm3.Lattice(w.nx, w.ny, w.sigma, w.tau, w.rho0, w.beta0, "fp32").init(w.rho).step(200)
            ref = L.densities()
            L.close()
            assert np.array_equal(rho, ref), (i, w.name)
    finally:
        lbm3.lbm3_batch_destroy(b)


def _classify_contacts(kind, rg, rb, gb, settled):
    """Checks of one instance's mixed-node counts (nodes where both fluids exceed 0.2) against
    its Neumann class.  Separate and kissing droplets share no interface (a kissing point
    contact leaves a few nodes: at most 3 % of the other interfaces), a partial-engulfing
    (Janus) droplet keeps all three interfaces, each at least 6 % of the longest (the shortest
    measured: 12.5 %, a Janus droplet whose junction angle in the matrix is 63 degrees).
    Once `settled`: complete engulfing leaves
    the engulfed droplet no contact with the matrix (<= 2 % of the engulfing droplet's), the
    critical engulfing state at most 15 %."""
    if kind in (morphology.SEPARATE, morphology.KISSING):
        return rg <= 0.03 * min(rb, gb)
    if kind == morphology.PARTIAL:
        return min(rg, rb, gb) >= 0.06 * max(rg, rb, gb)
    if not settled:
        return True
    if kind == morphology.ENGULF_1_BY_0:
        return gb <= 0.02 * rb and rg > 0
    if kind == morphology.ENGULF_0_BY_1:
        return rb <= 0.02 * gb and rg > 0
    if kind == morphology.CRITICAL_1_BY_0:
        return gb <= 0.15 * rb and rg > 0
    if kind == morphology.CRITICAL_0_BY_1:
        return rb <= 0.15 * gb and rg > 0
    raise ValueError(kind)


def test_morphology_sweep_64_instances():
    """The whole 8 x 8 sweep of the stability study (Sec. 4.1) as specified: 64 instances
    (sides 128-512, two tangent disks of radius side/6, sigma_gb = 0.01, ratios 0.25-2.0),
    FP32, one batch.  The Neumann inequalities give 38 partial-engulfing, 6 + 3
    complete-engulfing, 6 separate and 11 critical cases (4 kissing, 7 critical engulfing).
    After the study's 10 000 steps the separate, kissing and partial cases have their class
    (_classify_contacts); engulfing is still under way in the larger instances (capillary
    time of a radius-85 droplet ~ 1.5 x 10^4 steps).  After 100 000 steps every instance has
    its class, the critical engulfing states included."""
    from analysis import mixed_nodes
    ws = inputs.morphology_batch()
    kinds = [morphology.classify(*w.sigma) for w in ws]
    counts = {}
    for k in kinds:
        counts[k] = counts.get(k, 0) + 1
    assert counts == {morphology.PARTIAL: 38, morphology.ENGULF_1_BY_0: 3, morphology.ENGULF_0_BY_1: 6,
                      morphology.SEPARATE: 6, morphology.CRITICAL_1_BY_0: 3, morphology.CRITICAL_0_BY_1: 4,
                      morphology.KISSING: 4}
    b = _make_batch(ws, "fp32")
    bad = []
    try:
        done = 0
        for steps, settled in ((10000, False), (100000, True)):
            lbm3.lbm3_batch_step(b, steps - done)
            done = steps
            for i, w in enumerate(ws):
                obs, rho = _batch_state(b, i, w)
                assert obs["nonfinite"] == 0 and obs["step"] == steps
                rg, rb, gb = mixed_nodes(rho, 0, 1), mixed_nodes(rho, 0, 2), mixed_nodes(rho, 1, 2)
                ok = _classify_contacts(kinds[i], rg, rb, gb, settled)
                print("step %6d #%2d side %3d r12 %.2f r13 %.2f %-30s rg %5d rb %5d gb %5d %s" %
                      (steps, i, w.nx, w.meta["r12"], w.meta["r13"], kinds[i], rg, rb, gb, "" if ok else "FAIL"))
                if not ok:
                    bad.append((steps, i, kinds[i], rg, rb, gb))
    finally:
        lbm3.lbm3_batch_destroy(b)
    assert not bad, bad
