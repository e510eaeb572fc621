"""Writes janus256_fd.json: central finite differences (h = 1e-6) of the loss
L = sum_x (rho_1(x, T) - rho*(x))^2 for the 256^2 Janus droplet (two half-disks of radius
40, sigma = (0.006, 0.010, 0.012), tau = 0.8, T = 5000) with respect to the three
interfacial tensions and to four initial densities, computed with the FP64 oracle only.

    python tests/golden/make_adjoint_fd.py [--steps T]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1808_08555_amd import inputs  # noqa: E402

ENTRIES = [(0, 128, 90), (0, 100, 127), (1, 128, 166), (2, 128, 170)]  # (fluid, y, x)


def loss(p, rho0, target, steps):
    f = oracle.run(p, oracle.init(p, rho0), steps)
    r1 = f[0].sum(axis=0)
    return float(((r1 - target) ** 2).sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--h", type=float, default=1e-6)
    ap.add_argument("--out", default=os.path.join(HERE, "janus256_fd.json"))
    args = ap.parse_args()
    w = inputs.janus_halves(256, 40.0, (0.006, 0.010, 0.012), (0.8, 0.8, 0.8), args.steps)
    target = inputs.loss_target(w.rho[0], seed=5550)
    h = args.h
    t0 = time.time()
    base = oracle.Params(256, 256, w.sigma, w.tau)
    L0 = loss(base, w.rho, target, args.steps)
    dsig = []
    for q in range(3):
        vals = []
        for s in (+1, -1):
            sig = list(w.sigma)
            sig[q] += s * h
            vals.append(loss(oracle.Params(256, 256, tuple(sig), w.tau), w.rho, target, args.steps))
        dsig.append((vals[0] - vals[1]) / (2 * h))
        print(f"dL/dsigma[{q}] = {dsig[-1]:.10e}  ({time.time() - t0:.0f} s)", flush=True)
    drho = []
    for (k, y, x) in ENTRIES:
        vals = []
        for s in (+1, -1):
            r = w.rho.copy()
            r[k, y, x] += s * h
            vals.append(loss(base, r, target, args.steps))
        drho.append([k, y, x, (vals[0] - vals[1]) / (2 * h)])
        print(f"dL/drho0[{k},{y},{x}] = {drho[-1][3]:.10e}  ({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": "janus_halves(256, R=40), sigma=(0.006, 0.010, 0.012), tau=0.8, target seed 5550",
           "steps": args.steps, "h": h, "loss": L0, "dL_dsigma": dsig, "dL_drho0": drho,
           "oracle_threads": oracle.num_threads()}
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
