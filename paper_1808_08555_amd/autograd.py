"""Reverse-mode differentiation of a ternary colour-gradient run through torch.autograd.

``ternary_run(sigma, rho0, steps, ...)`` runs ``steps`` FP64 steps of the fused step from
the initial densities ``rho0`` (fluids at rest, f_{i,k} = w_i rho_k) with the interfacial
tensions ``sigma`` (order rg, rb, gb) and returns rho_1(x, T), the density of the first
fluid after the last step.  Its backward is the library's hand-written adjoint (reverse of
streaming, recolouring of Eq. 13 with the segregation law of Eqs. 18-20, collision with Guo
forcing of Eqs. 8-9, the interfacial force of Eq. 7 and the colour gradient of Eq. 12),
replayed from checkpoints taken every ``ckpt_every`` steps; it yields dL/dsigma (3,) and
dL/drho0 (3, ny, nx).

Both inputs are float64 tensors on any device; they cross the C ABI as host arrays, and
the gradients come back on the device of the corresponding input.  Every step of the
forward and reverse sweeps runs in the HIP library: there is no other implementation here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lbm3


def _host(t: torch.Tensor) -> np.ndarray:
    return np.ascontiguousarray(t.detach().to("cpu", torch.float64).numpy())


class TernaryRun(torch.autograd.Function):
    """rho_1(T) as a function of (sigma, rho0); non-tensor arguments are constants."""

    @staticmethod
    def forward(ctx, sigma, rho0, steps, ckpt_every, tau, rho_pure, beta0):
        if rho0.dim() != 3 or rho0.shape[0] != 3:
            raise ValueError(f"rho0 must be (3, ny, nx), got {tuple(rho0.shape)}")
        if sigma.shape != (3,):
            raise ValueError(f"sigma must be (3,), got {tuple(sigma.shape)}")
        ny, nx = int(rho0.shape[1]), int(rho0.shape[2])
        s = tuple(float(v) for v in _host(sigma))
        # the library's work is ordered on torch's current stream of the input's device (the
        # stream contract of the binding); on a CPU tensor, on the current device's
        dev = rho0.device if rho0.device.type == "cuda" else torch.device("cuda", torch.cuda.current_device())
        stream = torch.cuda.current_stream(dev)
        lat = lbm3.Lattice(nx, ny, s, tuple(tau), tuple(rho_pure), beta0, "fp64", stream=stream)
        lat.init(_host(rho0))
        lbm3.lbm3_adjoint_record(lat.h, steps, ckpt_every)
        rho_T = lat.densities()
        ctx.lattice = lat
        ctx.devices = (sigma.device, rho0.device)
        return torch.from_numpy(np.ascontiguousarray(rho_T[0])).to(rho0.device)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_rho1):
        lat = ctx.lattice
        if lat is None:
            raise RuntimeError("ternary_run: backward called twice (the tape is released after "
                               "the first reverse sweep)")
        ds, dr = lbm3.lbm3_adjoint(lat.h, _host(grad_rho1), lat.nx, lat.ny)
        lat.close()
        ctx.lattice = None
        dsig = torch.from_numpy(ds).to(ctx.devices[0]) if ctx.needs_input_grad[0] else None
        drho = torch.from_numpy(dr).to(ctx.devices[1]) if ctx.needs_input_grad[1] else None
        return dsig, drho, None, None, None, None, None


def ternary_run(sigma: torch.Tensor, rho0: torch.Tensor, steps: int, ckpt_every: int | None = None,
                tau=(1.0, 1.0, 1.0), rho_pure=(1.0, 1.0, 1.0), beta0: float = 0.7) -> torch.Tensor:
    """rho_1(x, T) after ``steps`` FP64 steps; differentiable in ``sigma`` and ``rho0``.
    ``ckpt_every`` must divide ``steps`` (default: the largest divisor not above 100)."""
    steps = int(steps)
    if ckpt_every is None:
        ckpt_every = max(d for d in range(1, min(steps, 100) + 1) if steps % d == 0) if steps else 1
    return TernaryRun.apply(sigma, rho0, steps, int(ckpt_every), tuple(tau), tuple(rho_pure),
                            float(beta0))
