"""ctypes wrapper of the C oracle (test infrastructure only).

Every function takes and returns float64 numpy arrays in the layout
W[v, j, i] (x fastest, contiguous). The status codes mirror the oracle's:
0 ok, -1 invalid argument, -3 CFL check failed, -4 non-finite or
non-physical state, -5 unsupported.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import build as _build

ADV, EULER, SPRAY = 0, 1, 2
PERIODIC, TRANSMISSIVE, DIRICHLET = 0, 1, 2
OK, EINVAL, ECFL, ENONFINITE, EUNSUPPORTED = 0, -1, -3, -4, -5
NVAR = {ADV: 1, EULER: 4, SPRAY: 6}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("model", C.c_int), ("bc", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int), ("npx", C.c_int), ("npy", C.c_int),
        ("lx", C.c_double), ("ly", C.c_double),
        ("gamma", C.c_double), ("ax", C.c_double), ("ay", C.c_double),
        ("K", C.c_double), ("theta", C.c_double), ("s_eps", C.c_double),
        ("cfl", C.c_double), ("dt_max", C.c_double),
        ("ghost", (C.c_double * 6) * 4),  # Dirichlet: west, east, south, north
        ("closure", C.c_int),  # spray: 0 lognormal fit, 1 entropy maximiser
    ]


def params(model: int, nx: int, ny: int, *, bc: int = PERIODIC, npx: int = 1,
           npy: int = 1, lx: float = 1.0, ly: float = 1.0, gamma: float = 1.4,
           ax: float = 0.0, ay: float = 0.0, K: float = 1.0, theta: float = 0.1,
           s_eps: float = 0.01, cfl: float = 0.45, dt_max: float = 0.0,
           ghost=None, closure: int = 0) -> Params:
    """ghost: Dirichlet states, 4 x nVar (west, east, south, north);
    closure: the spray's n(S=0), m_{-1/2} from a lognormal fit (0) or the
    entropy maximiser (1)."""
    P = Params(model, bc, nx, ny, npx, npy, lx, ly, gamma, ax, ay, K, theta,
               s_eps, cfl, dt_max)
    P.closure = closure
    if ghost is not None:
        g = np.asarray(ghost, dtype=np.float64)
        for side in range(4):
            for v in range(g.shape[1]):
                P.ghost[side][v] = g[side, v]
    return P


def from_preset(p, **over) -> Params:
    """Oracle parameters from a workload preset (any object with the preset's
    attribute names)."""
    kw = dict(bc=p.bc, npx=p.npart_x, npy=p.npart_y, lx=p.lx, ly=p.ly,
              gamma=p.gamma, ax=p.ax, ay=p.ay, K=p.K, theta=p.theta,
              s_eps=p.s_eps, cfl=p.cfl, dt_max=p.dt_max)
    kw.update(over)
    nx = kw.pop("nx", p.nx)
    ny = kw.pop("ny", p.ny)
    return params(p.model, nx, ny, **kw)


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        P = C.POINTER(Params)
        sig = {
            "orc_nvar": (C.c_int, [C.c_int]),
            "orc_validate": (C.c_int, [P]),
            "orc_phys_flux": (None, [P, _D, C.c_int, _D, _D]),
            "orc_num_flux": (None, [P, _D, _D, C.c_int, _D]),
            "orc_cell_speeds": (C.c_int, [P, _D, _D, _D]),
            "orc_spray_closure": (C.c_int, [P, _D, _D, _D]),
            "orc_maxent": (C.c_int, [_D, _D, _D, _D]),
            "orc_spray_source": (None, [P, _D, _D, _D]),
            "orc_set_threads": (None, [C.c_int]),
            "orc_get_threads": (C.c_int, []),
            "orc_cfl": (C.c_int, [P, _D, _D, _D, _D]),
            "orc_run": (C.c_int, [P, _D, _D, C.c_int, _D]),
            "orc_run_dts": (C.c_int, [P, _D, _D, C.c_int, _D]),
            "orc_step_fixed": (C.c_int, [P, _D, _D, C.c_double]),
            "orc_adjoint_step": (C.c_int, [P, _D, _D, C.c_double, _D, _D]),
            "orc_adjoint_run": (C.c_int, [P, _D, _D, C.c_int, _D, _D]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check_state(P: Params, W) -> np.ndarray:
    W = _f64(W)
    want = (NVAR[P.model], P.ny, P.nx)
    if W.shape != want:
        raise ValueError(f"state shape {W.shape} != {want}")
    return W


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def validate(P: Params) -> int:
    return int(lib().orc_validate(C.byref(P)))


def phys_flux(P: Params, w, d: int):
    w = _f64(w)
    f = np.zeros(NVAR[P.model])
    s = C.c_double()
    lib().orc_phys_flux(C.byref(P), _ptr(w), d, _ptr(f), C.byref(s))
    return f, s.value


def num_flux(P: Params, wl, wr, d: int) -> np.ndarray:
    wl, wr = _f64(wl), _f64(wr)
    f = np.zeros(NVAR[P.model])
    lib().orc_num_flux(C.byref(P), _ptr(wl), _ptr(wr), d, _ptr(f))
    return f


def cell_speeds(P: Params, w):
    w = _f64(w)
    sx, sy = C.c_double(), C.c_double()
    bad = lib().orc_cell_speeds(C.byref(P), _ptr(w), C.byref(sx), C.byref(sy))
    return int(bad), sx.value, sy.value


def spray_closure(P: Params, w):
    w = _f64(w)
    mmh, n0 = C.c_double(), C.c_double()
    rc = lib().orc_spray_closure(C.byref(P), _ptr(w), C.byref(mmh), C.byref(n0))
    if rc:
        raise OracleError(-4, "spray_closure")
    return mmh.value, n0.value


def maxent(m):
    """The entropy maximiser n(S) = exp(sum_k lam_k S^{k/2}) on [0, 1] with
    fractional moments m = (m_0, m_{1/2}, m_{2/2}, m_{3/2}): returns
    (lam, m_{-1/2}, n(S=0)); raises if the moments cannot be matched."""
    m = _f64(m)
    lam = np.zeros(4)
    mmh, n0 = C.c_double(), C.c_double()
    if lib().orc_maxent(_ptr(m), _ptr(lam), C.byref(mmh), C.byref(n0)):
        raise OracleError(-4, "maxent")
    return lam, mmh.value, n0.value


def spray_source(P: Params, w, ug) -> np.ndarray:
    w, ug = _f64(w), _f64(ug)
    S = np.zeros(6)
    lib().orc_spray_source(C.byref(P), _ptr(w), _ptr(ug), _ptr(S))
    return S


def cfl(P: Params, W):
    """Speed maxima (Sx, Sy) and the adaptive dt of state W."""
    W = _check_state(P, W)
    sx, sy, dt = C.c_double(), C.c_double(), C.c_double()
    rc = lib().orc_cfl(C.byref(P), _ptr(W), C.byref(sx), C.byref(sy), C.byref(dt))
    if rc:
        raise OracleError(rc, "cfl")
    return sx.value, sy.value, dt.value


def run(P: Params, W, nsteps: int, ug=None, *, return_status: bool = False):
    """nsteps adaptive steps; returns (W_n, dts)."""
    W = _check_state(P, W).copy()
    ugp = None if ug is None else _f64(ug)
    dts = np.zeros(max(nsteps, 1))
    rc = lib().orc_run(C.byref(P), _ptr(W), _ptr(ugp), int(nsteps), _ptr(dts))
    if return_status:
        return rc, W, dts[:nsteps]
    if rc:
        raise OracleError(rc, "run")
    return W, dts[:nsteps]


def run_dts(P: Params, W, dts, ug=None) -> np.ndarray:
    """Steps with the given time steps (no CFL logic)."""
    W = _check_state(P, W).copy()
    dts = _f64(dts).reshape(-1)
    ugp = None if ug is None else _f64(ug)
    rc = lib().orc_run_dts(C.byref(P), _ptr(W), _ptr(ugp), int(dts.size), _ptr(dts))
    if rc:
        raise OracleError(rc, "run_dts")
    return W


def step_fixed(P: Params, W, dt: float, ug=None):
    """One fixed-dt step with the paper's CFL check; returns (status, W)."""
    W = _check_state(P, W).copy()
    ugp = None if ug is None else _f64(ug)
    rc = lib().orc_step_fixed(C.byref(P), _ptr(W), _ptr(ugp), float(dt))
    return int(rc), W


def adjoint_step(P: Params, W, dt: float, lam, ug=None) -> np.ndarray:
    """(dW^{n+1}/dW^n)^T lam at state W (ug: the spray's gas velocity)."""
    W = _check_state(P, W)
    lam = _check_state(P, lam)
    out = np.empty_like(lam)
    ugp = None if ug is None else _f64(ug)
    rc = lib().orc_adjoint_step(C.byref(P), _ptr(W), _ptr(ugp), float(dt), _ptr(lam),
                                _ptr(out))
    if rc:
        raise OracleError(rc, "adjoint_step")
    return out


def adjoint_run(P: Params, W0, dts, lamN, ug=None) -> np.ndarray:
    """dL/dW^0 from dL/dW^N for len(dts) steps with frozen dts."""
    W0 = _check_state(P, W0)
    lam = _check_state(P, lamN).copy()
    dts = _f64(dts).reshape(-1)
    ugp = None if ug is None else _f64(ug)
    rc = lib().orc_adjoint_run(C.byref(P), _ptr(W0), _ptr(ugp), int(dts.size), _ptr(dts),
                               _ptr(lam))
    if rc:
        raise OracleError(rc, "adjoint_run")
    return lam


def dx_dy(P: Params):
    return P.lx / P.nx, P.ly / P.ny


def is_finite_state(W) -> bool:
    return bool(np.all(np.isfinite(W)))

