"""ctypes access to the three-dimensional oracle (lbm3_oracle3d.c): the ternary step on the
D3Q19 or the D3Q27 lattice in plain FP64.  TEST INFRASTRUCTURE ONLY: used by the test suite, never by the
product path.  The library is compiled from lbm3_oracle3d.c together with lbm3_oracle.c,
whose segregation law and local relaxation time it calls."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import Params, _d

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "lbm3_oracle.c"), os.path.join(_HERE, "lbm3_oracle3d.c")]
_LIB = os.path.join(_HERE, "liblbm3_oracle3d.so")
_lib = None
_DP = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS)
    if force or stale:
        tmp = f"{_LIB}.{os.getpid()}.tmp"  # one per process: parallel test workers may build at once
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        "-Wall", "-Wextra", "-Wno-unused-parameter", *_SRCS, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        from . import Problem
        PP = ctypes.POINTER(Problem)
        sigs = {
            "oracle3d_lattice": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _DP]),
            "oracle3d_init": (ctypes.c_int, [PP, ctypes.c_int32, ctypes.c_int32, _DP, _DP]),
            "oracle3d_step": (ctypes.c_int, [PP, ctypes.c_int32, ctypes.c_int32, _DP, _DP]),
            "oracle3d_run": (ctypes.c_int, [PP, ctypes.c_int32, ctypes.c_int32, _DP, ctypes.c_int64]),
            "oracle3d_observables": (ctypes.c_int, [PP, ctypes.c_int32, ctypes.c_int32, _DP, _DP]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def lattice(q: int = 19):
    """(e [q, 3], w [q]) of the oracle's link order (q = 19 or 27; D3Q19 is the first 19
    links of D3Q27)."""
    e = (ctypes.c_int32 * (3 * q))()
    w = (ctypes.c_double * q)()
    if lib().oracle3d_lattice(q, e, w):
        raise ValueError(f"q must be 19 or 27 (got {q})")
    return np.array(e[:], dtype=int).reshape(q, 3), np.array(w[:])


def init(p: Params, nz: int, rho: np.ndarray, q: int = 19) -> np.ndarray:
    """f_{i,k} = w_i rho_k; rho [3, nz, ny, nx] -> f [3, q, nz, ny, nx]."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    assert rho.shape == (3, nz, p.ny, p.nx)
    f = np.zeros((3, q, nz, p.ny, p.nx))
    if lib().oracle3d_init(ctypes.byref(p.c()), nz, q, _d(rho), _d(f)):
        raise ValueError(f"q must be 19 or 27 (got {q})")
    return f


def _q(f: np.ndarray) -> int:
    return int(f.shape[1])


def step(p: Params, nz: int, f: np.ndarray) -> np.ndarray:
    """One step of the state f [3, q, nz, ny, nx] (q from its shape)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    if lib().oracle3d_step(ctypes.byref(p.c()), nz, _q(f), _d(f), _d(out)):
        raise MemoryError("oracle3d_step")
    return out


def run(p: Params, nz: int, f: np.ndarray, nsteps: int) -> np.ndarray:
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    if lib().oracle3d_run(ctypes.byref(p.c()), nz, _q(f), _d(f), int(nsteps)):
        raise MemoryError("oracle3d_run")
    return f


def observables(p: Params, nz: int, f: np.ndarray) -> dict:
    out = np.zeros(8)
    f = np.ascontiguousarray(f, dtype=np.float64)
    if lib().oracle3d_observables(ctypes.byref(p.c()), nz, _q(f), _d(f), _d(out)):
        raise MemoryError("oracle3d_observables")
    return {"mass": out[0:3].copy(), "momentum": out[3:6].copy(), "kinetic_energy": out[6], "u_max": out[7]}


def source_text() -> str:
    with open(_SRCS[1]) as fh:
        return fh.read()


def compile_source(src_text: str, out_path: str) -> str:
    """Compile a three-dimensional oracle source text (with lbm3_oracle.c) with the flags of
    ``build``."""
    c_path = out_path + ".c"
    with open(c_path, "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    _SRCS[0], c_path, "-o", out_path, "-lm"], check=True)
    return out_path


class use_library:
    """Context manager: route the module's calls to another build (planted-mistake tests)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = lib()
        L = ctypes.CDLL(self.path)
        for name in ("oracle3d_lattice", "oracle3d_init", "oracle3d_step", "oracle3d_run",
                     "oracle3d_observables"):
            src, dst = getattr(self._saved, name), getattr(L, name)
            dst.restype, dst.argtypes = src.restype, src.argtypes
        _lib = L
        return L

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False
