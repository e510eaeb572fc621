"""Throughput of the fused ternary colour-gradient LBM step on one MI355X.

Prints ONE JSON line.  The headline ``value`` is the plain FP64 step in MLUPS (million
lattice-node updates per second) on the 4096^2 droplet-tiling workload, with inputs
resident in HBM; extra fields report the FP32-storage / FP32 variants, the batched
morphology sweep and the adjoint step, the HBM roofline of the dominant kernel and the
FP64 CPU oracle timed on the host as a reported baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline: plain FP64 vs FP32 batched vs adjoint step"
HBM_PEAK_GBS = 8000.0
# Bytes of the state of one node between steps: every precision keeps the recoloured state
# factored (f_dag_i, c_k, V_0, V_1: 16 values), in FP64 or FP32.  A launch reads and writes
# the state once, whether it advances one step or two.
STATE_BYTES = {"fp64": 16 * 8, "fp32_storage": 16 * 4, "fp32": 16 * 4}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(files=("lbm3_step_impl.h", "lbm3_rounding.h", "lbm3_tiles_f64.hip", "lbm3_internal.h")) -> str:
    """Hash of the kernel sources a profile summary was taken from (the 2D step's by
    default; the D3Q19 form's summaries use its own source)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1808_08555_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_figure(kernel_tag: str, kind: str, key: str):
    """The first `key: value` figure of the committed rocprofv3 summary
    profiles/<kernel_tag>_<kind>.txt, if that summary was taken from the current kernel
    source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_{kind}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(re.escape(key) + r":\s*([0-9.eE+]+)", text)
    files = ("lbm3d.hip", "lbm3_rounding.h") if kernel_tag.startswith("lbm3d") else None
    current = kernel_source_hash(files) if files else kernel_source_hash()
    if not m or not t or m.group(1) != current:
        return None
    return float(t.group(1))


def measured_traffic(kernel_tag: str):
    """HBM bytes per launch from the committed PMC summary (FETCH_SIZE, WRITE_SIZE)."""
    return profile_figure(kernel_tag, "pmc", "hbm_bytes_per_launch")


def time_steps(torch, lbm3, L, steps: int, reps: int = 3):
    """Median over reps of the time of `steps` steps, HIP events on the library's stream."""
    st = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        L.step(steps)
        b.record(st)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    return float(np.median(times))


def copy_bandwidth(torch, lbm3, nbytes: int = 2 << 30, reps: int = 5) -> float:
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    st = torch.cuda.current_stream()
    lbm3.lbm3_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, st)
    best = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        lbm3.lbm3_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, st)
        b.record(st)
        torch.cuda.synchronize()
        best.append(a.elapsed_time(b) / 1e3)
    del src, dst
    return 2 * nbytes / float(np.median(best)) / 1e9


def bench_plain(torch, lbm3, w, precision: str, steps: int, warmup: int, steps_per_launch: int = 0,
                beta_law: str = "paper", forcing: str = "guo"):
    """Times `steps` steps (even, so that two-step launches cover them all when used).
    Returns MLUPS and the dominant kernel's algorithmic bandwidth: state bytes read and
    written per launch over the time per launch."""
    st = torch.cuda.current_stream()
    L = lbm3.Lattice(w.nx, w.ny, w.sigma, w.tau, precision=precision, stream=st, beta_law=beta_law,
                     forcing=forcing)
    L.init(w.rho)
    L.set_steps_per_launch(steps_per_launch)
    L.step(warmup + (warmup % 2 == 0))  # leaves the state factored after an odd first step
    torch.cuda.synchronize()
    t = time_steps(torch, lbm3, L, steps)
    per_launch, t2, wg2 = lbm3.lbm3_get_pair_launch(L.h)
    tile = {"one_step": list(L.tile()), "steps_per_launch": per_launch}
    if per_launch == 2:
        tile["two_step"] = {"threads": t2, "workgroups": wg2}
    obs = L.observables()[0]
    L.close()
    n = w.nx * w.ny
    launches = steps // per_launch
    bytes_per_launch = 2 * STATE_BYTES[precision] * n
    return {"mlups": n * steps / t / 1e6, "ms_per_step": t / steps * 1e3, "tile": tile,
            "steps_per_launch": per_launch, "bytes_per_launch": bytes_per_launch,
            "ms_per_launch": t / launches * 1e3,
            "gbs": bytes_per_launch * launches / t / 1e9, "nonfinite": obs["nonfinite"]}


def bench_batched(torch, lbm3, inputs, steps: int):
    """The 64-instance morphology sweep (sides from {128..512}, FP32) advanced by graph
    launches; baselines: the plain FP32 step on one square lattice of the same node count,
    and the same 64 instances stepped with one launch per instance per step."""
    from paper_1808_08555_amd import autotune

    ws = inputs.morphology_batch()
    nodes = sum(w.nx * w.ny for w in ws)
    ps = [lbm3.make_params(w.nx, w.ny, w.sigma, w.tau, precision="fp32") for w in ws]
    st = torch.cuda.Stream()
    b = lbm3.lbm3_batch_create(ps, st)
    for i, w in enumerate(ws):
        lbm3.lbm3_batch_init_fields(b, i, w.rho)
    with torch.cuda.stream(st):
        # tuned afresh on every run (force): a cached plan from another run is not re-measured
        threads, rows = autotune.tune_batch(b, [w.nx for w in ws], "fp32", steps=40, force=True)
        lbm3.lbm3_batch_step(b, 40)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record(st)
        lbm3.lbm3_batch_step(b, steps)
        e.record(st)
        torch.cuda.synchronize()
    t = a.elapsed_time(e) / 1e3
    per_launch, t2, rows2, _ = lbm3.lbm3_batch_get_pair_launch(b)
    lbm3.lbm3_batch_destroy(b)
    res = {"instances": len(ws), "nodes": nodes, "mlups": nodes * steps / t / 1e6,
           "ms_per_step": t / steps * 1e3,
           "gbs": 2 * STATE_BYTES["fp32"] * nodes * steps / per_launch / t / 1e9,
           "steps_per_launch": per_launch, "one_step": {"threads": threads,
                                                        "rows_by_side": {str(k): v for k, v in rows.items()}}}
    if per_launch == 2:
        res["two_step"] = {"threads": t2, "rows": rows2}
    side = int(round(nodes ** 0.5))
    weq = inputs.droplet_tiling(side - side % 256 if side >= 512 else side, cell=256)
    res["plain_equal_nodes"] = bench_plain(torch, lbm3, weq, "fp32", steps, 20)["mlups"]
    # one launch per instance per step
    cur = torch.cuda.current_stream()
    Ls = [lbm3.Lattice(w.nx, w.ny, w.sigma, w.tau, precision="fp32", stream=cur).init(w.rho)
          for w in ws]
    seq_steps = max(10, steps // 20)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    a.record(cur)
    for _ in range(seq_steps):
        for L in Ls:
            L.step(1)
    e.record(cur)
    torch.cuda.synchronize()
    ts = a.elapsed_time(e) / 1e3
    for L in Ls:
        L.close()
    res["per_instance_launches"] = nodes * seq_steps / ts / 1e6
    return res


def bench_adjoint(torch, lbm3, inputs, n: int, steps: int, every: int):
    """Adjoint of the FP64 step on an n x n Janus droplet: forward with checkpoints, then the
    reverse sweep (segment recompute + reverse steps), each timed on the host around the
    blocking calls.  Adjoint MLUPS = nodes x steps / reverse-sweep time."""
    import time as _t
    R = 40.0 * n / 256.0
    w = inputs.janus_halves(n, R, (0.006, 0.010, 0.012), (0.8, 0.8, 0.8), steps)
    target = inputs.loss_target(w.rho[0], seed=5550)
    L = lbm3.Lattice(n, n, w.sigma, w.tau).init(w.rho)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    lbm3.lbm3_adjoint_record(L.h, steps, every)
    rho_T = L.densities()
    t1 = _t.perf_counter()
    lbm3.lbm3_adjoint(L.h, 2.0 * (rho_T[0] - target), n, n)
    t2 = _t.perf_counter()
    L.close()
    nodes = n * n
    return {"workload": f"Janus droplet {n}x{n}, R={R:g}, FP64, {steps} steps, checkpoint every {every}",
            "adjoint_mlups": round(nodes * steps / (t2 - t1) / 1e6, 1),
            "forward_with_checkpoints_mlups": round(nodes * steps / (t1 - t0) / 1e6, 1),
            "bytes_per_lu_stated": 1080,
            "frac_of_peak": round(1080 * nodes * steps / (t2 - t1) / 1e9 / HBM_PEAK_GBS, 4),
            "reverse_s": round(t2 - t1, 3), "forward_s": round(t1 - t0, 3)}


def bench_d3q19(torch, lbm3, inputs, n: int, steps: int, precision: str = "fp64", q: int = 19):
    """The three-dimensional form (D3Q19, or D3Q27 with q = 27) on an n^3 lattice of two
    tangent spheres, timed with HIP events on the lattice's stream.  Algorithmic bytes: the 3q
    populations read and written once per update (D3Q19 912 B in FP64, 456 B in FP32 or FP32
    storage; D3Q27 1296 B and 648 B)."""
    st = torch.cuda.current_stream()
    c = (n - 1) / 2
    R = n / 8.0
    rho = inputs.spheres(n, n, n, [(0, c - R, c, c, R), (1, c + R, c, c, R)])
    L = lbm3.Lattice3D(n, n, n, (0.01, 0.01, 0.01), (1.0, 1.0, 1.0), stream=st, precision=precision,
                       q=q).init(rho)
    L.step(5)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    L.step(steps)
    b.record(st)
    torch.cuda.synchronize()
    t = a.elapsed_time(b) / 1e3
    L.close()
    lu = n ** 3 * steps
    b = 2 * 3 * q * (8 if precision == "fp64" else 4)
    res = {"workload": f"D3Q{q} {n}^3, two tangent spheres of radius {R:g}, {precision}, {steps} steps",
           "mlups": round(lu / t / 1e6, 1), "bytes_per_lu_stated": b,
           "frac_of_peak": round(b * lu / t / 1e9 / HBM_PEAK_GBS, 4), "kernel": "k3_march (one launch per step)"}
    if n == 128 and precision == "fp64":
        # counters of the committed summary, if taken from the current source
        tag = f"lbm3d_d3q{q}_128"
        res["traffic_over_algorithmic"] = profile_figure(tag, "pmc", "traffic_over_algorithmic")
        res["valu_issue_frac"] = profile_figure(tag, "pmc", "VALU issue fraction")
    return res


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_mlups(oracle, w, steps: int):
    p = oracle.Params(w.nx, w.ny, w.sigma, w.tau)
    f = oracle.init(p, w.rho)
    t0 = time.perf_counter()
    oracle.run(p, f, steps)
    dt = time.perf_counter() - t0
    return w.nx * w.ny * steps / dt / 1e6, dt


def cpu_baseline(w, inputs):
    """The FP64 oracle on the host: the headline lattice (5 steps of 4096^2), the 256^2
    compound droplet (1000 steps) and the 1024^2 double droplet (100 steps) with OpenMP over
    rows on every core the process may use, and the 256^2 droplet (100 steps) on one thread
    (the oracle as written is serial per row)."""
    import oracle

    threads = oracle.num_threads()
    w256 = inputs.compound_droplet(256, 30.0, 60.0, 0.01, 0.01)
    w1024 = inputs.double_droplet(1024, 100.0, 1.0, 1.0, steps=0)
    head, t_head = _oracle_mlups(oracle, w, 5)
    s256, t256 = _oracle_mlups(oracle, w256, 1000)
    s1024, t1024 = _oracle_mlups(oracle, w1024, 100)
    oracle.set_num_threads(1)
    try:
        one, t_one = _oracle_mlups(oracle, w256, 100)
    finally:
        oracle.set_num_threads(threads)
    return {"value": round(head, 2), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"5 FP64 steps of the full {w.nx}x{w.ny} droplet-tiling lattice ({t_head:.1f} s, "
                      f"OpenMP over rows on {threads} threads)",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "usable_cores": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "all_core_mlups": {"droplet_tiling_4096_5_steps": round(head, 2),
                               "compound_256_1000_steps": round(s256, 2),
                               "double_droplet_1024_100_steps": round(s1024, 2)},
            "single_thread_mlups": {"compound_256_100_steps": round(one, 3)},
            "seconds": round(t_head + t256 + t1024 + t_one, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-plain", action="store_true", help="time the headline workload only")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_storage", "fp32"],
                    help="with --only-plain: the precision timed on the headline workload (its own "
                         "JSON line unless fp64)")
    ap.add_argument("--only-d3q19", action="store_true", help="time the D3Q19 form only (its own JSON line)")
    ap.add_argument("--only-d3q27", action="store_true", help="time the D3Q27 form only (its own JSON line)")
    ap.add_argument("--only-batched", action="store_true", help="time the batched form only (its own JSON line)")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="time the adjoint on the 2048^2 Janus droplet only (its own JSON line)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the step, its batched form and its adjoint run on a "
              "single MI355X; multi-GPU runs are not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1808_08555_amd import inputs, lbm3

    torch.cuda.set_device(0)
    if args.only_batched:
        print(json.dumps({"batched_fp32": bench_batched(torch, lbm3, inputs, args.steps)}), flush=True)
        return
    if args.only_d3q19 or args.only_d3q27:
        q = 27 if args.only_d3q27 else 19
        res = bench_d3q19(torch, lbm3, inputs, 128, args.steps, q=q)
        # the copy kernel's counters calibrate a PMC run of this mode
        res["device_copy_gbs"] = round(copy_bandwidth(torch, lbm3), 1)
        print(json.dumps({f"d3q{q}_fp64": res}), flush=True)
        return
    if args.only_adjoint:
        res = bench_adjoint(torch, lbm3, inputs, 2048, 200, 20)
        res["device_copy_gbs"] = round(copy_bandwidth(torch, lbm3), 1)
        print(json.dumps({"adjoint_fp64": {"janus_2048": res}}), flush=True)
        return
    w = inputs.droplet_tiling(4096)
    args.steps += args.steps % 2
    if args.only_plain and args.precision != "fp64":
        # one reduced-precision path on the headline workload (profiling runs)
        res = bench_plain(torch, lbm3, w, args.precision, args.steps, args.warmup)
        res["frac_of_peak"] = round(res["gbs"] / HBM_PEAK_GBS, 4)
        res["device_copy_gbs"] = round(copy_bandwidth(torch, lbm3), 1)
        print(json.dumps({args.precision: res}), flush=True)
        return
    log(f"workload {w.name}: {w.nx}x{w.ny}, FP64, {args.warmup} warm-up + {args.steps} timed steps")
    main_res = bench_plain(torch, lbm3, w, "fp64", args.steps, args.warmup)
    log(f"fp64 {main_res}")
    one_step = bench_plain(torch, lbm3, w, "fp64", args.steps, args.warmup, steps_per_launch=1)
    log(f"fp64, one step per launch {one_step}")
    extra = {}
    if not args.only_plain:
        for prec in ("fp32_storage", "fp32"):
            extra[prec] = bench_plain(torch, lbm3, w, prec, args.steps, args.warmup)
            log(f"{prec} {extra[prec]}")
        w2 = inputs.compound_droplet(256, 30.0, 60.0, 0.01, 0.01)
        for prec in ("fp64", "fp32_storage"):
            extra[f"compound_256_{prec}"] = bench_plain(torch, lbm3, w2, prec, 2000, 100)
            log(f"compound 256 {prec} {extra[f'compound_256_{prec}']}")
        # the comparison segregation laws of Eqs. (15)-(17): the same kernels with other host
        # constants, on the headline workload
        laws = {law: bench_plain(torch, lbm3, w, "fp64", 100, 10, beta_law=law)
                for law in ("spencer", "leclaire", "constant")}
        log(f"beta laws {laws}")
        # the comparison forcing of Eqs. (4)-(5) on the headline workload and launch form
        pert = bench_plain(torch, lbm3, w, "fp64", 100, 10, forcing="perturbation")
        log(f"perturbation forcing {pert}")
        d3 = bench_d3q19(torch, lbm3, inputs, 128, 60)
        log(f"d3q19 {d3}")
        d3r = {prec: bench_d3q19(torch, lbm3, inputs, 128, 60, prec) for prec in ("fp32_storage", "fp32")}
        log(f"d3q19 reduced precision {d3r}")
        d27 = {prec: bench_d3q19(torch, lbm3, inputs, 128, 40, prec, q=27) for prec in ("fp64", "fp32_storage", "fp32")}
        log(f"d3q27 {d27}")
        batched = bench_batched(torch, lbm3, inputs, 1000)
        log(f"batched {batched}")
        adjoint = {"janus_256": bench_adjoint(torch, lbm3, inputs, 256, 5000, 100),
                   "janus_2048": bench_adjoint(torch, lbm3, inputs, 2048, 200, 20)}
        log(f"adjoint {adjoint}")
    copy_gbs = copy_bandwidth(torch, lbm3)
    log(f"device copy {copy_gbs:.0f} GB/s")

    n = w.nx * w.ny
    achieved = main_res["gbs"]
    traffic = measured_traffic("lbm3_step_fp64_R4096")
    # VALU issue fraction of the dominant kernel from the committed instruction counters
    valu = (profile_figure("lbm3_step_fp64_R4096", "pmc", "VALU issue fraction")
            if main_res["steps_per_launch"] == 2 else None)
    kernel = ("two steps per launch (k_tiles2w: one step per wave group)" if main_res["steps_per_launch"] == 2
              else "one step per launch (k_tiles)")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
                "bytes_per_launch": main_res["bytes_per_launch"],
                "lu_per_launch": n * main_res["steps_per_launch"],
                "ms_per_launch": round(main_res["ms_per_launch"], 4),
                "frac_of_device_copy": round(achieved / copy_gbs, 4), "device_copy_gbs": round(copy_gbs, 1),
                "valu_issue_frac": valu,
                "bytes_per_lu": main_res["bytes_per_launch"] / (n * main_res["steps_per_launch"]),
                # the same MLUPS against other byte counts per lattice update: the 27 FP64
                # populations read and written once (432 B: the count of a kernel that stores
                # the populations and runs one step per launch; this kernel stores a factored
                # state and fuses two steps, so it can exceed 1 against it), and the smallest
                # exact factored state (15 values: rho_3 and c_3 follow from the others; 120 B
                # per update in two-step launches)
                "frac_vs_27_populations_432B": round(main_res["mlups"] * 1e6 * 432 / 1e9 / HBM_PEAK_GBS, 4),
                "frac_vs_15_values_two_step_120B": round(main_res["mlups"] * 1e6 * 120 / 1e9 / HBM_PEAK_GBS, 4),
                "one_step_kernel": {"mlups": round(one_step["mlups"], 1), "gbs": round(one_step["gbs"], 1),
                                    "frac": round(one_step["gbs"] / HBM_PEAK_GBS, 4),
                                    "frac_of_device_copy": round(one_step["gbs"] / copy_gbs, 4)}}
    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline ...")
        cpu = cpu_baseline(w, inputs)
        log(f"cpu {cpu}")
    line = {
        "metric": METRIC, "value": round(main_res["mlups"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "droplet tiling 4096x4096 periodic D2Q9 (16x16 cells of two tangent "
                               "R=40 disks in fluid 3, interface noise seed 1808), sigma=0.01, tau=1",
                   "nx": w.nx, "ny": w.ny, "tile": main_res["tile"], "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    for k, v in extra.items():
        line[k] = {"mlups": round(v["mlups"], 1), "ms_per_step": round(v["ms_per_step"], 4),
                   "gbs": round(v["gbs"], 1), "tile": v["tile"],
                   "frac_of_peak": round(v["gbs"] / HBM_PEAK_GBS, 4)}
    if not args.only_plain:
        line["batched_fp32"] = {
            "workload": "64 instances, sides {128..512} (SplitMix64 seed 855), two tangent disks "
                        "of radius side/6, 8x8 grid of tension ratios, FP32, one graph launch "
                        "per 20 steps",
            "mlups": round(batched["mlups"], 1), "ms_per_step": round(batched["ms_per_step"], 4),
            "gbs": round(batched["gbs"], 1), "frac_of_peak": round(batched["gbs"] / HBM_PEAK_GBS, 4),
            "nodes": batched["nodes"], "steps_per_launch": batched["steps_per_launch"],
            "one_step": batched["one_step"], "two_step": batched.get("two_step"),
            "baseline_plain_fp32_equal_nodes_mlups": round(batched["plain_equal_nodes"], 1),
            "baseline_one_launch_per_instance_mlups": round(batched["per_instance_launches"], 1)}
        line["adjoint_fp64"] = adjoint
        line["d3q19_fp64"] = d3
        for prec, v in d3r.items():
            line[f"d3q19_{prec}"] = v
        for prec, v in d27.items():
            line[f"d3q27_{prec}"] = v
        line["beta_laws_fp64"] = {
            "workload": "the headline droplet tiling, FP64, 100 timed steps per law",
            **{law: {"mlups": round(v["mlups"], 1), "frac_of_peak": round(v["gbs"] / HBM_PEAK_GBS, 4)}
               for law, v in laws.items()}}
        line["perturbation_forcing_fp64"] = {
            "workload": "the headline droplet tiling, FP64, 100 timed steps",
            "mlups": round(pert["mlups"], 1), "frac_of_peak": round(pert["gbs"] / HBM_PEAK_GBS, 4),
            "steps_per_launch": pert["steps_per_launch"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
