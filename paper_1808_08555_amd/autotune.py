"""Measured choice of the fused step's launch shape.

A launch shape is (threads per workgroup, rows per segment); results of the step do not
depend on it (bitwise), only its speed does.  ``tune_lattice`` times candidate shapes on a
lattice of the requested size, ``tune_batch`` tunes a batch (the workgroup size for the
whole launch, then the rows of each size class by coordinate descent).  Results are cached
in a JSON file keyed by GPU architecture, precision and size(s); the path is
``$LBM3_AUTOTUNE_CACHE`` or ``~/.cache/lbm3/autotune.json``.
"""
from __future__ import annotations

import json
import os

from . import inputs, lbm3

THREADS = (64, 128, 256, 512)
ROWS = (0, 2, 4, 8, 16, 32, 64, 128, 256)


def cache_path() -> str:
    return os.environ.get("LBM3_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "lbm3", "autotune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key: str, value):
    data = _load()
    data[key] = value
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _arch(torch) -> str:
    return str(getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gpu")).split(":")[0]


def _time(torch, fn, steps: int) -> float:
    """Median of three timings (ms per step) of `steps` steps, after `steps` untimed ones: a
    batch re-captures its graph after a shape change, and that must not land in a timed run.
    Each run is bracketed by device-wide synchronisation and timed on the host, so the
    timing holds whichever stream the handle orders its work on (a batch created without a
    stream runs on a stream of its own, which events on torch's current stream would not
    bracket)."""
    import time
    fn(steps)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        fn(steps)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3 / steps)
    return sorted(ts)[1]


def _cell_fields(nx: int, ny: int):
    """Two touching disks per 256-node cell (the benchmark's droplet tiling), cropped/tiled."""
    import numpy as np
    cell = min(256, nx, ny)
    R = cell * 40.0 / 256.0
    base = [(0, cell / 2 - R, cell / 2, R), (1, cell / 2 + R, cell / 2, R)]
    rho_c = inputs.rho_from_labels(inputs.label_disks(cell, cell, base))
    reps = (-(-ny // cell), -(-nx // cell))
    return np.ascontiguousarray(np.tile(rho_c, (1,) + reps)[:, :ny, :nx])


def tune_lattice(nx: int, ny: int, precision: str = "fp64", steps: int = 20,
                 force: bool = False, verbose: bool = False):
    """Fastest (threads, rows) for an nx x ny lattice; rows 0 means the slot-fitted choice."""
    import torch
    key = f"lattice/{_arch(torch)}/{precision}/{nx}x{ny}"
    if not force:
        hit = _load().get(key)
        if hit:
            return tuple(hit["tile"])
    st = torch.cuda.current_stream()
    L = lbm3.Lattice(nx, ny, precision=precision, stream=st).init(_cell_fields(nx, ny))
    best = None
    for t in THREADS:
        for r in ROWS:
            if t - 4 > 4 * nx and t > 64:
                continue
            L.set_tile(t, r)
            ms = _time(torch, L.step, steps)
            if verbose:
                print(f"  {precision} {nx}x{ny} threads={t} rows={L.tile()[1]}: {ms:.4f} ms/step")
            if best is None or ms < best[0]:
                best = (ms, t, r)
    L.close()
    _store(key, {"tile": [best[1], best[2]], "ms_per_step": best[0]})
    return best[1], best[2]


def tune_batch(batch, sizes, precision: str, steps: int = 20, force: bool = False,
               verbose: bool = False):
    """Tunes a batch handle in place: threads for the whole one-step launch, then rows per
    size class, then whether two steps per launch (the two-step pass on its own plan) beat
    one.  ``sizes`` lists the instances' nx (size classes are its distinct values).  Returns
    (threads, {side: rows}); the chosen steps per launch is set on the handle
    (lbm3_batch_get_pair_launch reads it back)."""
    import torch
    classes = sorted(set(int(s) for s in sizes))
    key = f"batch3/{_arch(torch)}/{precision}/" + ",".join(f"{s}" for s in sorted(int(s) for s in sizes))
    hit = None if force else _load().get(key)
    if hit:
        t = int(hit["threads"])
        lbm3.lbm3_batch_set_tile(batch, 0, t, 0)
        rows = {int(k): int(v) for k, v in hit["rows"].items()}
        for s, r in rows.items():
            lbm3.lbm3_batch_set_tile(batch, s, t, r)
        lbm3.lbm3_batch_set_steps_per_launch(batch, int(hit["steps_per_launch"]))
        return t, rows
    lbm3.lbm3_batch_set_steps_per_launch(batch, 1)

    def run(n):
        lbm3.lbm3_batch_step(batch, n)

    best_t, best_ms = None, None
    for t in THREADS:
        lbm3.lbm3_batch_set_tile(batch, 0, t, 0)
        for s in classes:
            lbm3.lbm3_batch_set_tile(batch, s, t, 0)
        ms = _time(torch, run, steps)
        if verbose:
            print(f"  batch threads={t} (automatic rows): {ms:.4f} ms/step")
        if best_ms is None or ms < best_ms:
            best_t, best_ms = t, ms
    lbm3.lbm3_batch_set_tile(batch, 0, best_t, 0)
    rows = {s: 0 for s in classes}
    for s in classes:
        lbm3.lbm3_batch_set_tile(batch, s, best_t, 0)
    for s in classes:
        for r in ROWS[1:]:
            lbm3.lbm3_batch_set_tile(batch, s, best_t, r)
            ms = _time(torch, run, steps)
            if verbose:
                print(f"  batch threads={best_t} side={s} rows={r}: {ms:.4f} ms/step")
            if ms < best_ms:
                best_ms, rows[s] = ms, r
        lbm3.lbm3_batch_set_tile(batch, s, best_t, rows[s])
    # two steps per launch: its width is the batch's threads (at most 256), tried on its own
    mode, final_t = 1, best_t
    lbm3.lbm3_batch_set_steps_per_launch(batch, 2)
    for t in (64, 128, 256):
        lbm3.lbm3_batch_set_tile(batch, 0, t, 0)
        if lbm3.lbm3_batch_get_pair_launch(batch)[0] != 2:
            continue
        ms = _time(torch, run, steps)
        if verbose:
            print(f"  batch two steps per launch, width {t}: {ms:.4f} ms/step")
        if ms < best_ms:
            best_ms, mode, final_t = ms, 2, t
    lbm3.lbm3_batch_set_steps_per_launch(batch, mode)
    lbm3.lbm3_batch_set_tile(batch, 0, final_t, 0)
    for s in classes:
        lbm3.lbm3_batch_set_tile(batch, s, final_t, rows[s])
    _store(key, {"threads": final_t, "rows": {str(k): v for k, v in rows.items()},
                 "steps_per_launch": mode, "ms_per_step": best_ms})
    return final_t, rows
