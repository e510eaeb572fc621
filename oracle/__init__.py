"""Plain FP64 CPU oracle of the ternary colour-gradient LBM step (arXiv:1808.08555).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only users.  The oracle is a plain C
library (``lbm3_oracle.c``) written from Sec. 2 of the paper; it shares no code
with the HIP library and never imports it.

Array layout everywhere: state ``f[3, 9, ny, nx]`` (post-streaming, x fastest),
densities ``rho[3, ny, nx]``, vectors ``[2, ny, nx]``.  Fluids 0, 1, 2 are the
paper's red, green, blue; ``sigma = (sigma_rg, sigma_rb, sigma_gb)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm3_oracle.c")
_LIB = os.path.join(_HERE, "liblbm3_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, IEEE double, no FMA contraction, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.{os.getpid()}.tmp"  # one per process: parallel test workers may build at once
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("rho0", ctypes.c_double * 3),
        ("sigma", ctypes.c_double * 3),
        ("tau", ctypes.c_double * 3),
        ("beta0", ctypes.c_double),
        ("beta_law", ctypes.c_int32),
        ("forcing", ctypes.c_int32),
    ]


# segregation laws: 0 the proposed law, Eqs. (18)-(20); the comparison laws of Eqs. (15)-(17)
BETA_LAWS = {"paper": 0, "spencer": 1, "leclaire": 2, "constant": 3}
# interfacial tension: the force of Eq. (7) with Guo's term, or the perturbation operator of Eqs. (4)-(5)
FORCINGS = {"guo": 0, "perturbation": 1}


@dataclass
class Params:
    nx: int
    ny: int
    sigma: tuple = (0.01, 0.01, 0.01)
    tau: tuple = (1.0, 1.0, 1.0)
    rho0: tuple = (1.0, 1.0, 1.0)
    beta0: float = 0.7
    beta_law: str = "paper"
    forcing: str = "guo"

    def c(self) -> Problem:
        p = Problem()
        p.nx, p.ny = int(self.nx), int(self.ny)
        for a in range(3):
            p.rho0[a] = float(self.rho0[a])
            p.sigma[a] = float(self.sigma[a])
            p.tau[a] = float(self.tau[a])
        p.beta0 = float(self.beta0)
        p.beta_law = BETA_LAWS[self.beta_law] if isinstance(self.beta_law, str) else int(self.beta_law)
        p.forcing = FORCINGS[self.forcing] if isinstance(self.forcing, str) else int(self.forcing)
        return p


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        PP = ctypes.POINTER(Problem)
        sig = {
            "oracle_lattice": (None, [_IP, _IP, _DP]),
            "oracle_X": (ctypes.c_double, [PP, ctypes.c_int, ctypes.c_int]),
            "oracle_g": (ctypes.c_double, [ctypes.c_double]),
            "oracle_beta": (ctypes.c_double, [PP, ctypes.c_int, ctypes.c_int, _DP]),
            "oracle_feq": (None, [ctypes.c_double] * 3 + [_DP]),
            "oracle_guo": (None, [ctypes.c_double] * 5 + [_DP]),
            "oracle_local_tau": (ctypes.c_double, [PP, _DP]),
            "oracle_collide_node": (None, [PP, _DP, _DP, ctypes.c_double, ctypes.c_double, _DP, _DP]),
            "oracle_recolour_node": (None, [PP, _DP, _DP, _DP, _DP, _DP]),
            "oracle_stress_node": (None, [PP, _DP, _DP, _DP, _DP]),
            "oracle_perturbation_node": (None, [PP, _DP, _DP, _DP, _DP]),
            "oracle_gradient": (None, [ctypes.c_int32, ctypes.c_int32, _DP, _DP, _DP]),
            "oracle_step": (ctypes.c_int, [PP, _DP, _DP]),
            "oracle_run": (ctypes.c_int, [PP, _DP, ctypes.c_int64]),
            "oracle_init": (None, [PP, _DP, _DP, _DP]),
            "oracle_fields": (ctypes.c_int, [PP, _DP, _DP, _DP, _DP, _DP]),
            "oracle_observables": (ctypes.c_int, [PP, _DP, _DP]),
            "oracle_step_nodes": (ctypes.c_int, [PP, _DP, ctypes.c_int32, _IP, _IP, _DP]),
            "oracle_num_threads": (ctypes.c_int, []),
            "oracle_set_num_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _vec(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64))


# ---------------------------------------------------------------- lattice / node pieces
def lattice():
    ex = (ctypes.c_int32 * 9)()
    ey = (ctypes.c_int32 * 9)()
    w = (ctypes.c_double * 9)()
    lib().oracle_lattice(ex, ey, w)
    return np.array(ex[:]), np.array(ey[:]), np.array(w[:])


def X(p: Params, k: int, l: int) -> float:
    return lib().oracle_X(ctypes.byref(p.c()), k, l)


def g(x: float) -> float:
    return lib().oracle_g(float(x))


def beta(p: Params, k: int, l: int, rho) -> float:
    r = _vec(rho)
    return lib().oracle_beta(ctypes.byref(p.c()), k, l, _d(r))


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().oracle_feq(rho, ux, uy, _d(out))
    return out


def guo(tau: float, ux: float, uy: float, Fx: float, Fy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().oracle_guo(tau, ux, uy, Fx, Fy, _d(out))
    return out


def local_tau(p: Params, rho) -> float:
    return lib().oracle_local_tau(ctypes.byref(p.c()), _d(_vec(rho)))


def collide_node(p: Params, rho_k, f, F):
    out = np.zeros(9)
    u = np.zeros(2)
    lib().oracle_collide_node(ctypes.byref(p.c()), _d(_vec(rho_k)), _d(_vec(f)), float(F[0]),
                              float(F[1]), _d(out), _d(u))
    return out, u


def recolour_node(p: Params, rho_k, gx, gy, fdag) -> np.ndarray:
    out = np.zeros(27)
    lib().oracle_recolour_node(ctypes.byref(p.c()), _d(_vec(rho_k)), _d(_vec(gx)), _d(_vec(gy)),
                               _d(_vec(fdag)), _d(out))
    return out.reshape(3, 9)


def stress_node(p: Params, rho_k, gx, gy) -> np.ndarray:
    out = np.zeros(4)
    lib().oracle_stress_node(ctypes.byref(p.c()), _d(_vec(rho_k)), _d(_vec(gx)), _d(_vec(gy)),
                             _d(out))
    return out


def perturbation_node(p: Params, rho_k, gx, gy) -> np.ndarray:
    """Phi_i of Eqs. (4)-(5) at one node (the comparison forcing)."""
    out = np.zeros(9)
    lib().oracle_perturbation_node(ctypes.byref(p.c()), _d(_vec(rho_k)), _d(_vec(gx)), _d(_vec(gy)),
                                   _d(out))
    return out


def gradient(phi: np.ndarray):
    phi = _vec(phi)
    ny, nx = phi.shape
    dx = np.zeros_like(phi)
    dy = np.zeros_like(phi)
    lib().oracle_gradient(nx, ny, _d(phi), _d(dx), _d(dy))
    return dx, dy


# ---------------------------------------------------------------- whole-grid calls
def init(p: Params, rho: np.ndarray, u: np.ndarray | None = None) -> np.ndarray:
    rho = _vec(rho)
    assert rho.shape == (3, p.ny, p.nx)
    f = np.zeros((3, 9, p.ny, p.nx))
    uu = None
    if u is not None:
        uu = _vec(u)
        assert uu.shape == (2, p.ny, p.nx)
    lib().oracle_init(ctypes.byref(p.c()), _d(rho), _d(uu) if uu is not None else None, _d(f))
    return f


def step(p: Params, f: np.ndarray) -> np.ndarray:
    f = _vec(f)
    out = np.empty_like(f)
    if lib().oracle_step(ctypes.byref(p.c()), _d(f), _d(out)):
        raise MemoryError("oracle_step")
    return out


def run(p: Params, f: np.ndarray, nsteps: int) -> np.ndarray:
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    if lib().oracle_run(ctypes.byref(p.c()), _d(f), int(nsteps)):
        raise MemoryError("oracle_run")
    return f


def fields(p: Params, f: np.ndarray):
    """Return (rho[3,ny,nx], u[2,ny,nx], F[2,ny,nx], tau[ny,nx])."""
    f = _vec(f)
    rho = np.zeros((3, p.ny, p.nx))
    u = np.zeros((2, p.ny, p.nx))
    F = np.zeros((2, p.ny, p.nx))
    tau = np.zeros((p.ny, p.nx))
    if lib().oracle_fields(ctypes.byref(p.c()), _d(f), _d(rho), _d(u), _d(F), _d(tau)):
        raise MemoryError("oracle_fields")
    return rho, u, F, tau


def observables(p: Params, f: np.ndarray) -> dict:
    out = np.zeros(7)
    if lib().oracle_observables(ctypes.byref(p.c()), _d(_vec(f)), _d(out)):
        raise MemoryError("oracle_observables")
    return {"mass": out[0:3].copy(), "momentum": out[3:5].copy(), "kinetic_energy": out[5],
            "u_max": out[6]}


def step_nodes(p: Params, f: np.ndarray, xs, ys) -> np.ndarray:
    """Post-streaming f after one step at nodes (xs[q], ys[q]); returns [count, 3, 9]."""
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    out = np.zeros((len(xs), 27))
    if lib().oracle_step_nodes(ctypes.byref(p.c()), _d(_vec(f)), len(xs),
                               xs.ctypes.data_as(_IP), ys.ctypes.data_as(_IP), _d(out)):
        raise MemoryError("oracle_step_nodes")
    return out.reshape(-1, 3, 9)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().oracle_set_num_threads(int(n))


def density(f: np.ndarray) -> np.ndarray:
    """rho_k = sum_i f_{i,k} of a state (text after the streaming equation)."""
    return f.sum(axis=1)


class use_library:
    """Context manager that points this module at another build of the oracle source
    (used by the tests that plant a mistake in a copy of the oracle and check that the
    pins catch it)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = lib()
        L = ctypes.CDLL(self.path)
        # copy the prototypes from the loaded default library
        for name in ("oracle_lattice", "oracle_X", "oracle_g", "oracle_beta", "oracle_feq",
                     "oracle_guo", "oracle_local_tau", "oracle_collide_node",
                     "oracle_recolour_node", "oracle_stress_node", "oracle_perturbation_node",
                     "oracle_gradient",
                     "oracle_step", "oracle_run", "oracle_init", "oracle_fields",
                     "oracle_observables", "oracle_step_nodes", "oracle_num_threads",
                     "oracle_set_num_threads"):
            src = getattr(self._saved, name)
            dst = getattr(L, name)
            dst.restype = src.restype
            dst.argtypes = src.argtypes
        _lib = L
        return L

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def compile_source(src_text: str, out_path: str) -> str:
    """Compile an oracle source text with the same flags as ``build``."""
    c_path = out_path + ".c"
    with open(c_path, "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    c_path, "-o", out_path, "-lm"], check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()
