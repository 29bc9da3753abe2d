"""ctypes front end of the FP64 oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_FIELDS = 3


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("nfields", ctypes.c_int32),
        ("expansion", ctypes.c_int32),
        ("L", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("lam", ctypes.c_double),
        ("G", ctypes.c_double * MAX_FIELDS),
        ("mu2", ctypes.c_double * MAX_FIELDS),
        ("kappa", ctypes.c_double),
    ]


class _State(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("tau", ctypes.c_double),
        ("a", ctypes.c_double),
        ("adot_half", ctypes.c_double),
        ("adot", ctypes.c_double),
        ("kin", ctypes.c_double * MAX_FIELDS),
        ("grad", ctypes.c_double * MAX_FIELDS),
        ("pot", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("mean", ctypes.c_double * MAX_FIELDS),
        ("mean_sq", ctypes.c_double * MAX_FIELDS),
        ("resid", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        assert lib.or_sizeof_params() == ctypes.sizeof(_Params)
        assert lib.or_sizeof_state() == ctypes.sizeof(_State)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        sp = ctypes.POINTER(_State)
        lib.or_laplacian.argtypes = [pp, dp, dp]
        lib.or_grad_energy.argtypes = [pp, dp]
        lib.or_grad_energy.restype = ctypes.c_double
        lib.or_mean_potential.argtypes = [pp, dp, ctypes.c_double]
        lib.or_mean_potential.restype = ctypes.c_double
        lib.or_potential_point.argtypes = [pp, dp, ctypes.c_double]
        lib.or_potential_point.restype = ctypes.c_double
        lib.or_dpotential_point.argtypes = [pp, dp, ctypes.c_double, ctypes.c_int32]
        lib.or_dpotential_point.restype = ctypes.c_double
        lib.or_solve_adot.argtypes = [ctypes.c_double] * 4
        lib.or_solve_adot.restype = ctypes.c_double
        lib.or_start.argtypes = [pp, dp, dp, dp, dp, sp]
        lib.or_step.argtypes = [pp, dp, dp, sp]
        lib.or_run.argtypes = [pp, dp, dp, sp, ctypes.c_int64, sp]
        _lib = lib
    return _lib


@dataclass
class OracleParams:
    """Physics and numerics of one lattice (program units)."""
    dims: int
    N: int
    nfields: int
    L: float
    dt: float
    lam: float = 1.0
    G: Sequence[float] = (0.0, 0.0, 0.0)
    mu2: Sequence[float] = (0.0, 0.0, 0.0)
    expansion: bool = False
    kappa: float = 0.0

    def c(self) -> _Params:
        G = list(self.G) + [0.0] * (MAX_FIELDS - len(self.G))
        mu2 = list(self.mu2) + [0.0] * (MAX_FIELDS - len(self.mu2))
        return _Params(self.dims, self.N, self.nfields, int(bool(self.expansion)),
                       float(self.L), float(self.dt), float(self.lam),
                       (ctypes.c_double * MAX_FIELDS)(*G[:MAX_FIELDS]),
                       (ctypes.c_double * MAX_FIELDS)(*mu2[:MAX_FIELDS]),
                       float(self.kappa))

    @property
    def shape(self):
        return (self.N,) * self.dims

    @property
    def nsites(self) -> int:
        return self.N ** self.dims


@dataclass
class OracleState:
    step: int
    tau: float
    a: float
    adot_half: float
    adot: float
    kin: List[float]
    grad: List[float]
    pot: float
    rho: float
    mean: List[float]
    mean_sq: List[float]
    resid: float

    @classmethod
    def from_c(cls, s: _State, nf: int) -> "OracleState":
        return cls(int(s.step), s.tau, s.a, s.adot_half, s.adot,
                   list(s.kin)[:nf], list(s.grad)[:nf], s.pot, s.rho,
                   list(s.mean)[:nf], list(s.mean_sq)[:nf], s.resid)


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One lattice evolved by the oracle.

    ``phi``/``phidot`` are the physical program-unit field and its derivative
    at tau = 0 (a = 1), shaped ``[nfields, N, ..., N]``.  After construction
    the object holds f^0, pi^{1/2}; each ``step`` advances by one leapfrog step.
    """

    def __init__(self, params: OracleParams, phi: np.ndarray, phidot: np.ndarray):
        self.params = params
        self._p = params.c()
        shape = (params.nfields,) + params.shape
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(shape)
        phidot = np.ascontiguousarray(phidot, dtype=np.float64).reshape(shape)
        self.f = np.empty(shape, np.float64)
        self.pi = np.empty(shape, np.float64)
        self._st = _State()
        _load().or_start(ctypes.byref(self._p), _dptr(phi), _dptr(phidot),
                         _dptr(self.f), _dptr(self.pi), ctypes.byref(self._st))
        self.log: List[OracleState] = [self.state]

    @property
    def state(self) -> OracleState:
        return OracleState.from_c(self._st, self.params.nfields)

    def step(self, n: int = 1, record: bool = True) -> OracleState:
        if n <= 0:
            return self.state
        if record:
            buf = (_State * n)()
            _load().or_run(ctypes.byref(self._p), _dptr(self.f), _dptr(self.pi),
                           ctypes.byref(self._st), n, buf)
            nf = self.params.nfields
            self.log.extend(OracleState.from_c(buf[k], nf) for k in range(n))
        else:
            _load().or_run(ctypes.byref(self._p), _dptr(self.f), _dptr(self.pi),
                           ctypes.byref(self._st), n, None)
        return self.state


def laplacian(params: OracleParams, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    p = params.c()
    _load().or_laplacian(ctypes.byref(p), _dptr(f), _dptr(out))
    return out


def grad_energy(params: OracleParams, f: np.ndarray) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    p = params.c()
    return _load().or_grad_energy(ctypes.byref(p), _dptr(f))


def mean_potential(params: OracleParams, f: np.ndarray, a: float) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    p = params.c()
    return _load().or_mean_potential(ctypes.byref(p), _dptr(f), float(a))


def potential_point(params: OracleParams, v: Sequence[float], a: float) -> float:
    arr = np.array(list(v) + [0.0] * (MAX_FIELDS - len(v)), np.float64)
    p = params.c()
    return _load().or_potential_point(ctypes.byref(p), _dptr(arr), float(a))


def dpotential_point(params: OracleParams, v: Sequence[float], a: float, i: int) -> float:
    arr = np.array(list(v) + [0.0] * (MAX_FIELDS - len(v)), np.float64)
    p = params.c()
    return _load().or_dpotential_point(ctypes.byref(p), _dptr(arr), float(a), int(i))


def solve_adot(a: float, y: float, S: float, dt: float) -> float:
    return _load().or_solve_adot(float(a), float(y), float(S), float(dt))
