"""ctypes binding of liblbm3.so (the HIP library), one Python function per C entry point.

The functions keep the C names and only marshal arguments: NumPy float64 arrays in
and out, a HIP stream handle (a ``torch.cuda.Stream``, its integer handle, or None for
the null stream).  Every step of the method runs in the library's HIP kernels; if the
library is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; LBM3_LIBRARY may name another build of the same sources
LIB_PATH = os.environ.get("LBM3_LIBRARY") or os.path.join(_HERE, "liblbm3.so")

LBM3_OK, LBM3_EINVAL, LBM3_ENOMEM, LBM3_EDEVICE, LBM3_EUNSUPPORTED, LBM3_ENONFINITE, \
    LBM3_ESTATE = 0, -1, -2, -3, -4, -5, -6
LBM3_FP64, LBM3_FP32_STORAGE, LBM3_FP32 = 0, 1, 2
LBM3_PERIODIC = 0
PRECISIONS = {"fp64": LBM3_FP64, "fp32_storage": LBM3_FP32_STORAGE, "fp32": LBM3_FP32}
# segregation laws: the paper's Eqs. (18)-(20) and the comparison laws of Eqs. (15)-(17)
LBM3_BETA_PAPER, LBM3_BETA_SPENCER, LBM3_BETA_LECLAIRE, LBM3_BETA_CONSTANT = 0, 1, 2, 3
BETA_LAWS = {"paper": LBM3_BETA_PAPER, "spencer": LBM3_BETA_SPENCER, "leclaire": LBM3_BETA_LECLAIRE,
             "constant": LBM3_BETA_CONSTANT}
# interfacial tension: the force of Eq. (7) with Guo's term, or the perturbation operator of Eqs. (4)-(5)
LBM3_FORCING_GUO, LBM3_FORCING_PERTURBATION = 0, 1
FORCINGS = {"guo": LBM3_FORCING_GUO, "perturbation": LBM3_FORCING_PERTURBATION}
ERROR_NAMES = {0: "LBM3_OK", -1: "LBM3_EINVAL", -2: "LBM3_ENOMEM", -3: "LBM3_EDEVICE",
               -4: "LBM3_EUNSUPPORTED", -5: "LBM3_ENONFINITE", -6: "LBM3_ESTATE"}


class lbm3_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("rho0", ctypes.c_double * 3), ("sigma", ctypes.c_double * 3),
        ("tau", ctypes.c_double * 3), ("beta0", ctypes.c_double),
        ("boundary", ctypes.c_int32), ("wall_wettability", ctypes.c_double * 3),
        ("precision", ctypes.c_int32), ("beta_law", ctypes.c_int32), ("forcing", ctypes.c_int32),
    ]


class lbm3d_obs(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("mass", ctypes.c_double * 3),
        ("momentum", ctypes.c_double * 3), ("kinetic_energy", ctypes.c_double),
        ("u_max", ctypes.c_double), ("nonfinite", ctypes.c_int32),
    ]


class lbm3_obs(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("mass", ctypes.c_double * 3),
        ("momentum", ctypes.c_double * 2), ("kinetic_energy", ctypes.c_double),
        ("u_max", ctypes.c_double), ("nonfinite", ctypes.c_int32),
    ]


class Lbm3Error(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} -> {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


def lib():
    """Load liblbm3.so from the package directory (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1808_08555_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(lbm3_params)
        H = ctypes.c_void_p
        I = ctypes.c_int
        protos = {
            "lbm3_create": (I, [P, _VP, ctypes.POINTER(H)]),
            "lbm3_init_fields": (I, [H, _DP, _DP]),
            "lbm3_set_state": (I, [H, _DP]),
            "lbm3_step": (I, [H, ctypes.c_int64]),
            "lbm3_observables": (I, [H, ctypes.POINTER(lbm3_obs), _DP, _DP]),
            "lbm3_observables_noalloc": (I, [H, ctypes.POINTER(lbm3_obs)]),
            "lbm3_destroy": (I, [H]),
            "lbm3_last_error": (ctypes.c_char_p, []),
            "lbm3_derived": (I, [P, _DP, _DP, _DP]),
            "lbm3_set_tile": (I, [H, ctypes.c_int32, ctypes.c_int32]),
            "lbm3_get_tile": (I, [H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
            "lbm3_set_steps_per_launch": (I, [H, ctypes.c_int32]),
            "lbm3_get_pair_launch": (I, [H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]),
            "lbm3_state_buffer": (I, [H, ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int32)]),
            "lbm3_batch_create": (I, [P, ctypes.c_int32, _VP, ctypes.POINTER(H)]),
            "lbm3_batch_init_fields": (I, [H, ctypes.c_int32, _DP, _DP]),
            "lbm3_batch_step": (I, [H, ctypes.c_int64]),
            "lbm3_batch_observables": (I, [H, ctypes.c_int32, ctypes.POINTER(lbm3_obs), _DP]),
            "lbm3_batch_set_tile": (I, [H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
            "lbm3_batch_set_steps_per_launch": (I, [H, ctypes.c_int32]),
            "lbm3_batch_get_pair_launch": (I, [H] + [ctypes.POINTER(ctypes.c_int32)] * 4),
            "lbm3_batch_destroy": (I, [H]),
            "lbm3_adjoint_record": (I, [H, ctypes.c_int64, ctypes.c_int32]),
            "lbm3_adjoint": (I, [H, _DP, _DP, _DP]),
            "lbm3_adjoint_pipeline_slots": (I, [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                                                ctypes.c_uint64]),
            "lbm3_device_copy": (I, [_VP, _VP, ctypes.c_int64, _VP]),
            "lbm3d_create": (I, [P, ctypes.c_int32, _VP, ctypes.POINTER(H)]),
            "lbm3d_create_lattice": (I, [P, ctypes.c_int32, ctypes.c_int32, _VP, ctypes.POINTER(H)]),
            "lbm3d_init_fields": (I, [H, _DP]),
            "lbm3d_step": (I, [H, ctypes.c_int64]),
            "lbm3d_observables": (I, [H, ctypes.POINTER(lbm3d_obs), _DP, _DP]),
            "lbm3d_destroy": (I, [H]),
        }
        for name, (res, args) in protos.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def lbm3_last_error() -> str:
    return lib().lbm3_last_error().decode()


def _check(rc: int, func: str):
    if rc != LBM3_OK:
        raise Lbm3Error(rc, func, lbm3_last_error())


def _dptr(a):
    if a is None:
        return None
    assert isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _stream_handle(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream: HIP stream under ROCm


def make_params(nx: int, ny: int, sigma=(0.01, 0.01, 0.01), tau=(1.0, 1.0, 1.0),
                rho0=(1.0, 1.0, 1.0), beta0: float = 0.7, precision="fp64",
                boundary: int = LBM3_PERIODIC, wall_wettability=(0.0, 0.0, 0.0),
                beta_law="paper", forcing="guo") -> lbm3_params:
    p = lbm3_params()
    p.nx, p.ny = int(nx), int(ny)
    for a in range(3):
        p.rho0[a] = float(rho0[a])
        p.sigma[a] = float(sigma[a])
        p.tau[a] = float(tau[a])
        p.wall_wettability[a] = float(wall_wettability[a])
    p.beta0 = float(beta0)
    p.boundary = int(boundary)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.beta_law = BETA_LAWS[beta_law] if isinstance(beta_law, str) else int(beta_law)
    p.forcing = FORCINGS[forcing] if isinstance(forcing, str) else int(forcing)
    return p


# ----------------------------------------------------------------- plain lattice
def lbm3_create(params: lbm3_params, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().lbm3_create(ctypes.byref(params), _stream_handle(stream), ctypes.byref(h)),
           "lbm3_create")
    return h


def lbm3_init_fields(h, rho: np.ndarray, u: np.ndarray | None = None):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    _check(lib().lbm3_init_fields(h, _dptr(rho), _dptr(u)), "lbm3_init_fields")


def lbm3_set_state(h, f: np.ndarray):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(lib().lbm3_set_state(h, _dptr(f)), "lbm3_set_state")


def lbm3_step(h, n: int):
    _check(lib().lbm3_step(h, int(n)), "lbm3_step")


def _obs_dict(o: lbm3_obs) -> dict:
    return {"step": int(o.step), "mass": np.array(o.mass[:]), "momentum": np.array(o.momentum[:]),
            "kinetic_energy": float(o.kinetic_energy), "u_max": float(o.u_max),
            "nonfinite": int(o.nonfinite)}


def lbm3_observables(h, nx: int, ny: int, want_rho: bool = False, want_f: bool = False,
                     raise_nonfinite: bool = True):
    """Returns (observables dict, rho[3,ny,nx] or None, f[3,9,ny,nx] or None)."""
    o = lbm3_obs()
    rho = np.empty((3, ny, nx)) if want_rho else None
    f = np.empty((3, 9, ny, nx)) if want_f else None
    rc = lib().lbm3_observables(h, ctypes.byref(o), _dptr(rho), _dptr(f))
    if rc != LBM3_OK and not (rc == LBM3_ENONFINITE and not raise_nonfinite):
        _check(rc, "lbm3_observables")
    return _obs_dict(o), rho, f


def lbm3_observables_noalloc(h, raise_nonfinite: bool = True) -> dict:
    """The observables of lbm3_observables (no densities or populations), computed with the
    library's static device scratch: the call allocates nothing."""
    o = lbm3_obs()
    rc = lib().lbm3_observables_noalloc(h, ctypes.byref(o))
    if rc != LBM3_OK and not (rc == LBM3_ENONFINITE and not raise_nonfinite):
        _check(rc, "lbm3_observables_noalloc")
    return _obs_dict(o)


def lbm3_destroy(h):
    if h is not None:
        _check(lib().lbm3_destroy(h), "lbm3_destroy")


def lbm3_derived(params: lbm3_params):
    X = (ctypes.c_double * 3)()
    g = (ctypes.c_double * 3)()
    nu = (ctypes.c_double * 3)()
    _check(lib().lbm3_derived(ctypes.byref(params), X, g, nu), "lbm3_derived")
    return np.array(X[:]), np.array(g[:]), np.array(nu[:])


def lbm3_set_tile(h, threads: int, rows: int):
    _check(lib().lbm3_set_tile(h, int(threads), int(rows)), "lbm3_set_tile")


def lbm3_set_steps_per_launch(h, mode: int):
    """0 = by lattice size, 1 = one step per launch, 2 = two steps per launch where possible."""
    _check(lib().lbm3_set_steps_per_launch(h, int(mode)), "lbm3_set_steps_per_launch")


def lbm3_get_pair_launch(h):
    """(steps per launch for pairs, threads, workgroups) of the launch used for pairs of steps."""
    st, th, wg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lbm3_get_pair_launch(h, ctypes.byref(st), ctypes.byref(th), ctypes.byref(wg)),
           "lbm3_get_pair_launch")
    return st.value, th.value, wg.value


def lbm3_get_tile(h):
    t = ctypes.c_int32()
    r = ctypes.c_int32()
    _check(lib().lbm3_get_tile(h, ctypes.byref(t), ctypes.byref(r)), "lbm3_get_tile")
    return t.value, r.value


def lbm3_state_buffer(h):
    """(device pointer, element bytes, plane stride, row pitch, planes) of the current state
    buffer: 27 planes of populations after init / set_state, 16 factored planes after a step."""
    p = ctypes.c_void_p()
    eb = ctypes.c_int32()
    pl = ctypes.c_int64()
    pt = ctypes.c_int64()
    nq = ctypes.c_int32()
    _check(lib().lbm3_state_buffer(h, ctypes.byref(p), ctypes.byref(eb), ctypes.byref(pl),
                                   ctypes.byref(pt), ctypes.byref(nq)), "lbm3_state_buffer")
    return p.value, eb.value, pl.value, pt.value, nq.value


def lbm3_device_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream=None):
    _check(lib().lbm3_device_copy(dst_ptr, src_ptr, int(nbytes), _stream_handle(stream)),
           "lbm3_device_copy")


# ----------------------------------------------------------------- batched form
def lbm3_batch_create(params_list, stream=None):
    arr = (lbm3_params * len(params_list))(*params_list)
    h = ctypes.c_void_p()
    _check(lib().lbm3_batch_create(arr, len(params_list), _stream_handle(stream), ctypes.byref(h)),
           "lbm3_batch_create")
    return h


def lbm3_batch_init_fields(b, idx: int, rho: np.ndarray, u: np.ndarray | None = None):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    _check(lib().lbm3_batch_init_fields(b, int(idx), _dptr(rho), _dptr(u)), "lbm3_batch_init_fields")


def lbm3_batch_step(b, n: int):
    _check(lib().lbm3_batch_step(b, int(n)), "lbm3_batch_step")


def lbm3_batch_observables(b, idx: int, nx: int, ny: int, want_rho: bool = False):
    o = lbm3_obs()
    rho = np.empty((3, ny, nx)) if want_rho else None
    _check(lib().lbm3_batch_observables(b, int(idx), ctypes.byref(o), _dptr(rho)),
           "lbm3_batch_observables")
    return _obs_dict(o), rho


def lbm3_batch_set_tile(b, side: int, threads: int, rows: int):
    _check(lib().lbm3_batch_set_tile(b, int(side), int(threads), int(rows)), "lbm3_batch_set_tile")


def lbm3_batch_set_steps_per_launch(b, mode: int):
    _check(lib().lbm3_batch_set_steps_per_launch(b, int(mode)), "lbm3_batch_set_steps_per_launch")


def lbm3_batch_get_pair_launch(b):
    """(steps per launch, threads, rows, workgroups) of the batch's launch for pairs of steps."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().lbm3_batch_get_pair_launch(b, *[ctypes.byref(x) for x in v]), "lbm3_batch_get_pair_launch")
    return tuple(x.value for x in v)


def lbm3_batch_destroy(b):
    if b is not None:
        _check(lib().lbm3_batch_destroy(b), "lbm3_batch_destroy")


# ----------------------------------------------------------------- adjoint
def lbm3_adjoint_record(h, nsteps: int, ckpt_every: int):
    _check(lib().lbm3_adjoint_record(h, int(nsteps), int(ckpt_every)), "lbm3_adjoint_record")


def lbm3_adjoint(h, drho1_T: np.ndarray, nx: int, ny: int):
    """Returns (dL/dsigma[3], dL/drho0[3, ny, nx])."""
    g = np.ascontiguousarray(drho1_T, dtype=np.float64)
    assert g.shape == (ny, nx)
    ds = np.zeros(3)
    dr = np.zeros((3, ny, nx))
    _check(lib().lbm3_adjoint(h, _dptr(g), _dptr(ds), _dptr(dr)), "lbm3_adjoint")
    return ds, dr


def lbm3_adjoint_pipeline_slots(nodes: int, ws_two_slots: int, ws_held: int, device_free: int) -> int:
    """Pipeline slots lbm3_adjoint uses (host rule, no device work): 2 or 1."""
    return int(lib().lbm3_adjoint_pipeline_slots(int(nodes), int(ws_two_slots), int(ws_held), int(device_free)))


# ----------------------------------------------------------------- convenience
@dataclass
class Lattice:
    """Owning wrapper around one lbm3 handle."""
    nx: int
    ny: int
    sigma: tuple = (0.01, 0.01, 0.01)
    tau: tuple = (1.0, 1.0, 1.0)
    rho0: tuple = (1.0, 1.0, 1.0)
    beta0: float = 0.7
    precision: str = "fp64"
    stream: object = None
    beta_law: str = "paper"
    forcing: str = "guo"

    def __post_init__(self):
        self.params = make_params(self.nx, self.ny, self.sigma, self.tau, self.rho0, self.beta0,
                                  self.precision, beta_law=self.beta_law, forcing=self.forcing)
        self.h = lbm3_create(self.params, self.stream)

    def init(self, rho, u=None):
        lbm3_init_fields(self.h, rho, u)
        return self

    def set_state(self, f):
        lbm3_set_state(self.h, f)
        return self

    def step(self, n: int = 1):
        lbm3_step(self.h, n)
        return self

    def observables(self, want_rho=False, want_f=False, raise_nonfinite=True):
        return lbm3_observables(self.h, self.nx, self.ny, want_rho, want_f, raise_nonfinite)

    def state(self) -> np.ndarray:
        return self.observables(want_f=True)[2]

    def densities(self) -> np.ndarray:
        return self.observables(want_rho=True)[1]

    def set_tile(self, threads: int, rows: int):
        lbm3_set_tile(self.h, threads, rows)
        return self

    def tile(self):
        return lbm3_get_tile(self.h)

    def set_steps_per_launch(self, mode: int):
        lbm3_set_steps_per_launch(self.h, mode)
        return self

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- D3Q19 form
class Lattice3D:
    """Owning wrapper around one lbm3d handle (the three-dimensional form, periodic; lattice
    q = 19 (D3Q19) or 27 (D3Q27); precision "fp64", "fp32_storage" or "fp32")."""

    def __init__(self, nx: int, ny: int, nz: int, sigma=(0.01, 0.01, 0.01), tau=(1.0, 1.0, 1.0),
                 rho0=(1.0, 1.0, 1.0), beta0: float = 0.7, beta_law="paper", stream=None,
                 precision: str = "fp64", q: int = 19):
        self.nx, self.ny, self.nz, self.q = int(nx), int(ny), int(nz), int(q)
        self.params = make_params(nx, ny, sigma, tau, rho0, beta0, precision, beta_law=beta_law)
        h = ctypes.c_void_p()
        _check(lib().lbm3d_create_lattice(ctypes.byref(self.params), self.nz, self.q, _stream_handle(stream),
                                          ctypes.byref(h)), "lbm3d_create_lattice")
        self.h = h

    def init(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        assert rho.shape == (3, self.nz, self.ny, self.nx)
        _check(lib().lbm3d_init_fields(self.h, _dptr(rho)), "lbm3d_init_fields")
        return self

    def step(self, n: int = 1):
        _check(lib().lbm3d_step(self.h, int(n)), "lbm3d_step")
        return self

    def observables(self, want_rho: bool = False, want_f: bool = False):
        """(dict, rho [3, nz, ny, nx] or None, f [3, q, nz, ny, nx] or None); blocking."""
        o = lbm3d_obs()
        shape = (self.nz, self.ny, self.nx)
        rho = np.empty((3,) + shape) if want_rho else None
        f = np.empty((3, self.q) + shape) if want_f else None
        _check(lib().lbm3d_observables(self.h, ctypes.byref(o), _dptr(rho), _dptr(f)), "lbm3d_observables")
        d = {"step": int(o.step), "mass": np.array(o.mass[:]), "momentum": np.array(o.momentum[:]),
             "kinetic_energy": float(o.kinetic_energy), "u_max": float(o.u_max), "nonfinite": int(o.nonfinite)}
        return d, rho, f

    def state(self) -> np.ndarray:
        return self.observables(want_f=True)[2]

    def densities(self) -> np.ndarray:
        return self.observables(want_rho=True)[1]

    def close(self):
        if self.h is not None:
            _check(lib().lbm3d_destroy(self.h), "lbm3d_destroy")
            self.h = None
