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
_SRCS = (_SRC, os.path.join(_HERE, "grf.c"))
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_FIELDS = 3


def build(force: bool = True) -> str:
    """Compile oracle.c and grf.c with gcc into liboracle.so next to them."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu99",
            "-fPIC", "-shared", "-o", tmp, *_SRCS, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


MAX_TERMS = 8


class _Term(ctypes.Structure):
    _fields_ = [("coef", ctypes.c_double), ("exp", ctypes.c_int32 * MAX_FIELDS), ("pad", ctypes.c_int32)]


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
        ("vacuum", ctypes.c_double),
        ("nterms", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("terms", _Term * MAX_TERMS),
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
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
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
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.or_philox4x64_10.argtypes = [u64p, u64p, u64p]
        lib.or_grf_normals.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, dp, dp]
        lib.or_grf_modes.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.or_grf_sites.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64), dp]
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
    vacuum: float = 0.0
    # user-defined polynomial potential, ((coef, (e0, e1, e2)), ...): when
    # given, V(phi) = sum coef phi0^e0 phi1^e1 phi2^e2 replaces lam, G, mu2, vacuum
    terms: Optional[Sequence] = None

    def c(self) -> _Params:
        G = list(self.G) + [0.0] * (MAX_FIELDS - len(self.G))
        mu2 = list(self.mu2) + [0.0] * (MAX_FIELDS - len(self.mu2))
        tarr = (_Term * MAX_TERMS)()
        nterms = 0
        if self.terms:
            nterms = len(self.terms)
            assert nterms <= MAX_TERMS
            for t, (coef, exps) in enumerate(self.terms):
                e = list(exps) + [0] * (MAX_FIELDS - len(exps))
                tarr[t] = _Term(float(coef), (ctypes.c_int32 * MAX_FIELDS)(*e[:MAX_FIELDS]), 0)
        return _Params(self.dims, self.N, self.nfields, int(bool(self.expansion)),
                       float(self.L), float(self.dt), float(self.lam),
                       (ctypes.c_double * MAX_FIELDS)(*G[:MAX_FIELDS]),
                       (ctypes.c_double * MAX_FIELDS)(*mu2[:MAX_FIELDS]),
                       float(self.kappa), float(self.vacuum), int(nterms), 0, tarr)

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


# ---- seeded Gaussian random fields (definition in grf.c) -------------------

FIELD, MOMENTUM = 0, 1


def philox4x64_10(counter: Sequence[int], key: Sequence[int]) -> List[int]:
    """One Philox4x64-10 block (four 64-bit words)."""
    c = (ctypes.c_uint64 * 4)(*[int(v) & (2 ** 64 - 1) for v in counter])
    k = (ctypes.c_uint64 * 2)(*[int(v) & (2 ** 64 - 1) for v in key])
    out = (ctypes.c_uint64 * 4)()
    _load().or_philox4x64_10(c, k, out)
    return list(out)


def grf_normals(seed: int, box_index: int, stream: int):
    X, Y = ctypes.c_double(), ctypes.c_double()
    _load().or_grf_normals(int(seed), int(box_index), int(stream), ctypes.byref(X), ctypes.byref(Y))
    return X.value, Y.value


def grf_mode_parts(seed: int, field: int, kind: int, dims: int, N: int, L: float, amp: float,
                   m_eff2: float):
    """(Re c_n, Im c_n) over the (2K+1)^dims box of wave vectors n_j in
    [-K, K], K = N/4, C order."""
    W = 2 * (N // 4) + 1
    re = np.empty((W,) * dims, np.float64)
    im = np.empty((W,) * dims, np.float64)
    _load().or_grf_modes(int(seed), int(field), int(kind), int(dims), int(N), float(L), float(amp),
                         float(m_eff2), _dptr(re), _dptr(im))
    return re, im


def grf_modes(seed: int, field: int, kind: int, dims: int, N: int, L: float, amp: float,
              m_eff2: float) -> np.ndarray:
    """c_n over the (2K+1)^dims box (complex)."""
    re, im = grf_mode_parts(seed, field, kind, dims, N, L, amp, m_eff2)
    return re + 1j * im


def grf_field(seed: int, field: int, kind: int, dims: int, N: int, L: float, amp: float,
              m_eff2: float) -> np.ndarray:
    """delta(x) = Re sum_n c_n exp(2 pi i n.x/N) on the whole grid, by one
    inverse FFT of the modes placed at n mod N (unnormalised sum)."""
    c = grf_modes(seed, field, kind, dims, N, L, amp, m_eff2)
    K = N // 4
    full = np.zeros((N,) * dims, np.complex128)
    idx = np.arange(-K, K + 1) % N
    full[np.ix_(*([idx] * dims))] = c
    return np.ascontiguousarray(np.real(np.fft.ifftn(full)) * float(N) ** dims)


def grf_sites(re: np.ndarray, im: np.ndarray, N: int, sites: np.ndarray) -> np.ndarray:
    """delta at the listed C-order sites, by direct summation over the modes
    (re, im as from grf_mode_parts)."""
    dims = re.ndim
    re = np.ascontiguousarray(re, dtype=np.float64)
    im = np.ascontiguousarray(im, dtype=np.float64)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty(sites.shape[0], np.float64)
    _load().or_grf_sites(dims, int(N), _dptr(re), _dptr(im), sites.shape[0],
                         sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(out))
    return out


def grf_initial(seed: int, dims: int, N: int, L: float, nfields: int, m_eff2: Sequence[float],
                amp: float = 1e-3, background: Sequence[float] = (1.0, 0.0, 0.0),
                background_dot: Sequence[float] = (0.0, 0.0, 0.0)):
    """(phi, phidot) [nfields, N, ..., N]: background plus delta per field."""
    shape = (nfields,) + (N,) * dims
    phi = np.empty(shape, np.float64)
    phidot = np.empty(shape, np.float64)
    for i in range(nfields):
        phi[i] = grf_field(seed, i, FIELD, dims, N, L, amp, m_eff2[i]) + background[i]
        phidot[i] = grf_field(seed, i, MOMENTUM, dims, N, L, amp, m_eff2[i]) + background_dot[i]
    return phi, phidot


# ---- radially binned power spectra ------------------------------------------

def spectrum_bins(dims: int, N: int) -> int:
    """floor(sqrt(dims) N / 2) + 1 bins."""
    import math
    return math.isqrt(dims * (N // 2) ** 2) + 1


def spectrum(g: np.ndarray):
    """(power, count) of one field array g (shape (N,)*dims): F(n) = N^-d
    sum_x g(x) e^{-2 pi i n.x/N}; power[j] = sum |F(n)|^2 over the integer
    wave vectors n (components in [-N/2, N/2)) with floor(|n|) = j, count[j]
    the number of them."""
    import math
    g = np.asarray(g, dtype=np.float64)
    dims, N = g.ndim, g.shape[0]
    F = np.fft.fftn(g) / float(N) ** dims
    n = np.fft.fftfreq(N, 1.0 / N).astype(np.int64)
    n2 = np.zeros((N,) * dims, np.int64)
    for d in range(dims):
        shape = [1] * dims
        shape[d] = N
        n2 = n2 + (n * n).reshape(shape)
    bins = np.array([math.isqrt(int(v)) for v in np.unique(n2)])
    lut = dict(zip(np.unique(n2).tolist(), bins.tolist()))
    b = np.vectorize(lut.get, otypes=[np.int64])(n2)
    nb = spectrum_bins(dims, N)
    power = np.bincount(b.ravel(), weights=(np.abs(F) ** 2).ravel(), minlength=nb)
    count = np.bincount(b.ravel(), minlength=nb).astype(np.float64)
    return power, count
