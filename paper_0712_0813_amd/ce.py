"""Thin ctypes binding of the C ABI in ``include/ce.h`` (same names).

Argument marshalling only: every step of the evolution runs in ``libce.so``'s
HIP kernels.  Loading fails loudly if the library has not been built.
PyTorch, when used, only supplies device memory (an arena) and a stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libce.so")
MAX_FIELDS = 3
ENERGY_LOG = 1024

CE_OK, CE_EINVAL, CE_ENOMEM, CE_EDEVICE, CE_ESTATE, CE_ENONFINITE, CE_EBUSY = 0, -1, -2, -3, -4, -5, -6
CE_FP32, CE_FP64 = 0, 1
CE_MODEL_QUARTIC, CE_MODEL_POLYNOMIAL = 0, 1

_STATUS_NAMES = {0: "CE_OK", -1: "CE_EINVAL", -2: "CE_ENOMEM", -3: "CE_EDEVICE", -4: "CE_ESTATE",
                 -5: "CE_ENONFINITE", -6: "CE_EBUSY"}


class CeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


MAX_TERMS, MAX_EXP, MAX_DEGREE = 8, 6, 8


class ce_term(ctypes.Structure):
    _fields_ = [("coef", ctypes.c_double), ("exp", ctypes.c_int32 * MAX_FIELDS), ("pad_", ctypes.c_int32)]


class ce_params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32), ("N", ctypes.c_int32), ("nfields", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("model", ctypes.c_int32), ("expansion", ctypes.c_int32),
        ("L", ctypes.c_double), ("dt", ctypes.c_double), ("lam", ctypes.c_double),
        ("G", ctypes.c_double * MAX_FIELDS), ("mu2", ctypes.c_double * MAX_FIELDS),
        ("kappa", ctypes.c_double), ("vacuum", ctypes.c_double),
        ("nterms", ctypes.c_int32), ("pad_", ctypes.c_int32), ("terms", ce_term * MAX_TERMS),
        ("stream", ctypes.c_void_p), ("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
    ]


CE_KERNEL_DIRECT, CE_KERNEL_TILED3D, CE_KERNEL_STREAM2D = 0, 1, 2


class ce_launch(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("sites_per_thread", ctypes.c_int32),
                ("lanes_per_row", ctypes.c_int32), ("block", ctypes.c_int32),
                ("planes", ctypes.c_int32), ("grid", ctypes.c_int32)]

    def as_tuple(self):
        return (self.kernel, self.sites_per_thread, self.lanes_per_row, self.block, self.planes,
                self.grid)


# tiled shapes the library builds: (sites_per_thread, lanes_per_row, block)
TILED_SHAPES = ((4, 16, 256), (4, 8, 256), (2, 32, 256), (2, 32, 512), (2, 16, 256), (2, 16, 512),
                (4, 64, 256), (4, 64, 512))


class ce_energy(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("tau", ctypes.c_double), ("a", ctypes.c_double),
        ("adot", ctypes.c_double), ("hubble", ctypes.c_double),
        ("kin", ctypes.c_double * MAX_FIELDS), ("grad", ctypes.c_double * MAX_FIELDS),
        ("pot", ctypes.c_double), ("rho", ctypes.c_double),
        ("mean", ctypes.c_double * MAX_FIELDS), ("mean_sq", ctypes.c_double * MAX_FIELDS),
        ("friedmann_residual", ctypes.c_double), ("nonfinite", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]

    def as_dict(self, nfields: int = MAX_FIELDS) -> dict:
        return {
            "step": int(self.step), "tau": self.tau, "a": self.a, "adot": self.adot,
            "hubble": self.hubble, "kin": list(self.kin)[:nfields],
            "grad": list(self.grad)[:nfields], "pot": self.pot, "rho": self.rho,
            "mean": list(self.mean)[:nfields], "mean_sq": list(self.mean_sq)[:nfields],
            "friedmann_residual": self.friedmann_residual, "nonfinite": int(self.nonfinite),
        }


class ce_init_spec(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("amp", ctypes.c_double),
                ("background", ctypes.c_double * MAX_FIELDS), ("background_dot", ctypes.c_double * MAX_FIELDS),
                ("m_eff2", ctypes.c_double * MAX_FIELDS)]


def make_init_spec(seed: int, m_eff2: Sequence[float], amp: float = 1e-3,
                   background: Sequence[float] = (1.0, 0.0, 0.0),
                   background_dot: Sequence[float] = (0.0, 0.0, 0.0)) -> ce_init_spec:
    def pad(v):
        v = [float(x) for x in v][:MAX_FIELDS]
        return (ctypes.c_double * MAX_FIELDS)(*(v + [0.0] * (MAX_FIELDS - len(v))))
    return ce_init_spec(int(seed), float(amp), pad(background), pad(background_dot), pad(m_eff2))


def lattice_init_spec(lat) -> ce_init_spec:
    """The device-generation spec of a workloads.Lattice (its seed, amplitude,
    backgrounds and effective masses)."""
    return make_init_spec(lat.seed, lat.m_eff2(), lat.amp, lat.background)


class ce_image_header(ctypes.Structure):
    _fields_ = [
        ("magic", ctypes.c_char * 8), ("version", ctypes.c_uint32), ("header_bytes", ctypes.c_uint32),
        ("dims", ctypes.c_int32), ("N", ctypes.c_int32), ("nfields", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("model", ctypes.c_int32), ("expansion", ctypes.c_int32),
        ("L", ctypes.c_double), ("dt", ctypes.c_double), ("lam", ctypes.c_double),
        ("G", ctypes.c_double * MAX_FIELDS), ("mu2", ctypes.c_double * MAX_FIELDS),
        ("kappa", ctypes.c_double), ("step", ctypes.c_int64), ("launch", ce_launch),
        ("state_bytes", ctypes.c_uint64), ("ring_bytes", ctypes.c_uint64),
        ("field_bytes", ctypes.c_uint64), ("total_bytes", ctypes.c_uint64),
        ("vacuum", ctypes.c_double), ("nterms", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("terms", ce_term * MAX_TERMS), ("reserved", ctypes.c_uint8 * 120),
    ]


IMAGE_MAGIC = b"CEGRID\0\1"
IMAGE_VERSION = 2


class ce_pool_info(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("used_bytes", ctypes.c_size_t),
                ("members", ctypes.c_int32), ("active", ctypes.c_int32), ("classes", ctypes.c_int32),
                ("admitting", ctypes.c_int32), ("steps_run", ctypes.c_int64)]


# every symbol include/ce.h declares, with its ctypes signature
_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "ce_required_bytes": ([ctypes.POINTER(ce_params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ce_create": ([ctypes.POINTER(ce_params), ctypes.POINTER(_P)], ctypes.c_int),
    "ce_load_fields": ([_P, ctypes.c_int32, ctypes.c_int32, _DP, _DP], ctypes.c_int),
    "ce_generate_fields": ([_P, ctypes.POINTER(ce_init_spec)], ctypes.c_int),
    "ce_generate_fields_noalloc": ([_P, ctypes.POINTER(ce_init_spec)], ctypes.c_int),
    "ce_step": ([_P, ctypes.c_int64], ctypes.c_int),
    "ce_energies": ([_P, ctypes.POINTER(ce_energy)], ctypes.c_int),
    "ce_energy_log": ([_P, ctypes.c_int32, ctypes.POINTER(ce_energy)], ctypes.c_int),
    "ce_read_fields": ([_P, _DP, _DP], ctypes.c_int),
    "ce_read_sites": ([_P, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _DP, _DP],
                      ctypes.c_int),
    "ce_get_step": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ce_set_step_block": ([_P, ctypes.c_int32], ctypes.c_int),
    "ce_get_launch": ([_P, ctypes.POINTER(ce_launch)], ctypes.c_int),
    "ce_set_launch": ([_P, ctypes.POINTER(ce_launch)], ctypes.c_int),
    "ce_sync": ([_P], ctypes.c_int),
    "ce_time_steps": ([_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "ce_destroy": ([_P], None),
    "ce_spectrum_bins": ([_P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "ce_spectrum": ([_P, ctypes.c_int32, _DP, _DP, _DP], ctypes.c_int),
    "ce_image_bytes": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ce_save_image": ([_P, _P, ctypes.c_size_t], ctypes.c_int),
    "ce_image_params": ([_P, ctypes.c_size_t, ctypes.POINTER(ce_params)], ctypes.c_int),
    "ce_restore_image": ([_P, _P, ctypes.c_size_t], ctypes.c_int),
    "ce_pool_create": ([ctypes.c_size_t, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "ce_pool_admit": ([_P, ctypes.POINTER(ce_params), _DP, _DP, ctypes.c_int64,
                       ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ce_pool_admit_with_launch": ([_P, ctypes.POINTER(ce_params), ctypes.POINTER(ce_launch), _DP, _DP,
                                   ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ce_pool_admit_generated": ([_P, ctypes.POINTER(ce_params), ctypes.POINTER(ce_launch),
                                 ctypes.POINTER(ce_init_spec), ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
                                ctypes.c_int),
    "ce_pool_launch_for": ([ctypes.POINTER(ce_params), ctypes.POINTER(ce_launch)], ctypes.c_int),
    "ce_pool_run_block": ([_P, ctypes.c_int32], ctypes.c_int),
    "ce_pool_set_member_launch": ([_P, ctypes.c_int64, ctypes.POINTER(ce_launch)], ctypes.c_int),
    "ce_pool_poll": ([_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ce_energy)],
                     ctypes.c_int),
    "ce_pool_steps_left": ([_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ce_pool_set_quota": ([_P, ctypes.c_int64, ctypes.c_int64], ctypes.c_int),
    "ce_pool_retire": ([_P, ctypes.c_int64, _DP, _DP], ctypes.c_int),
    "ce_pool_get_info": ([_P, ctypes.POINTER(ce_pool_info)], ctypes.c_int),
    "ce_pool_member_image_bytes": ([_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ce_pool_save_member": ([_P, ctypes.c_int64, _P, ctypes.c_size_t], ctypes.c_int),
    "ce_pool_admit_image": ([_P, _P, ctypes.c_size_t, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
                            ctypes.c_int),
    "ce_pool_destroy": ([_P], None),
    "ce_stream_copy": ([_P, _P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                        ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "ce_stream_probe": ([ctypes.c_int32, _P, _P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                         ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "ce_last_error": ([], ctypes.c_char_p),
}

_lib = None


def load_library() -> ctypes.CDLL:
    """Load libce.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_0712_0813_amd.build`")
        # Load order only: PyTorch ships its own HIP runtime, and once this
        # library's runtime has initialised the GPU in a process, torch
        # imported afterwards reports no GPU.  Importing torch (when it is
        # installed) before the library keeps both usable in one process,
        # as they are when torch supplies device memory and streams.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def ce_last_error() -> str:
    return load_library().ce_last_error().decode()


def _check(status: int, what: str, allow=()) -> int:
    if status != CE_OK and status not in allow:
        raise CeError(status, f"{what}: {ce_last_error()}")
    return status


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_DP)


def make_params(dims: int, N: int, nfields: int, L: float, dt: float, *, lam: float = 1.0,
                G: Sequence[float] = (0.0, 0.0, 0.0), mu2: Sequence[float] = (0.0, 0.0, 0.0),
                expansion: bool = False, kappa: float = 0.0, precision: int = CE_FP32,
                stream: Optional[int] = None, arena: Optional[int] = None,
                arena_bytes: int = 0, vacuum: float = 0.0, terms=None) -> ce_params:
    """Run parameters.  With `terms` (a sequence of (coef, (e0, e1, e2))) the
    model is CE_MODEL_POLYNOMIAL, V(phi) = sum coef phi0^e0 phi1^e1 phi2^e2,
    and lam, G, mu2 and vacuum must be left at zero."""
    G = list(G) + [0.0] * (MAX_FIELDS - len(G))
    mu2 = list(mu2) + [0.0] * (MAX_FIELDS - len(mu2))
    model, nterms = CE_MODEL_QUARTIC, 0
    tarr = (ce_term * MAX_TERMS)()
    if terms is not None:
        model, nterms = CE_MODEL_POLYNOMIAL, len(terms)
        for t, (coef, exps) in enumerate(list(terms)[:MAX_TERMS]):
            e = list(exps) + [0] * (MAX_FIELDS - len(exps))
            tarr[t] = ce_term(float(coef), (ctypes.c_int32 * MAX_FIELDS)(*e[:MAX_FIELDS]), 0)
    return ce_params(dims, N, nfields, precision, model, int(bool(expansion)),
                     float(L), float(dt), float(lam),
                     (ctypes.c_double * MAX_FIELDS)(*G[:MAX_FIELDS]),
                     (ctypes.c_double * MAX_FIELDS)(*mu2[:MAX_FIELDS]), float(kappa), float(vacuum),
                     int(nterms), 0, tarr, stream, arena, int(arena_bytes))


def ce_required_bytes(params: ce_params) -> int:
    out = ctypes.c_size_t()
    _check(load_library().ce_required_bytes(ctypes.byref(params), ctypes.byref(out)), "ce_required_bytes")
    return out.value


def ce_create(params: ce_params) -> int:
    h = ctypes.c_void_p()
    _check(load_library().ce_create(ctypes.byref(params), ctypes.byref(h)), "ce_create")
    return h.value


def ce_load_fields(sim: int, first: int, phi: np.ndarray, phidot: np.ndarray) -> None:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    phidot = np.ascontiguousarray(phidot, dtype=np.float64)
    count = phi.shape[0]
    if phidot.shape != phi.shape:
        raise ValueError("phi and phidot shapes differ")
    _check(load_library().ce_load_fields(sim, first, count, _dptr(phi), _dptr(phidot)), "ce_load_fields")


def ce_generate_fields(sim: int, spec: ce_init_spec) -> None:
    _check(load_library().ce_generate_fields(sim, ctypes.byref(spec)), "ce_generate_fields")


def ce_generate_fields_noalloc(sim: int, spec: ce_init_spec) -> None:
    _check(load_library().ce_generate_fields_noalloc(sim, ctypes.byref(spec)), "ce_generate_fields_noalloc")


def ce_step(sim: int, nsteps: int) -> None:
    _check(load_library().ce_step(sim, int(nsteps)), "ce_step")


def ce_energies(sim: int, allow_nonfinite: bool = False) -> ce_energy:
    e = ce_energy()
    allow = (CE_ENONFINITE,) if allow_nonfinite else ()
    _check(load_library().ce_energies(sim, ctypes.byref(e)), "ce_energies", allow)
    return e


def ce_energy_log(sim: int, count: int):
    buf = (ce_energy * count)()
    _check(load_library().ce_energy_log(sim, int(count), buf), "ce_energy_log")
    return list(buf)


def ce_read_fields(sim: int, nfields: int, shape, want_f: bool = True, want_fdot: bool = True):
    f = np.empty((nfields,) + tuple(shape), np.float64) if want_f else None
    fd = np.empty((nfields,) + tuple(shape), np.float64) if want_fdot else None
    _check(load_library().ce_read_fields(sim, _dptr(f), _dptr(fd)), "ce_read_fields")
    return f, fd


def ce_read_sites(sim: int, field: int, sites: np.ndarray):
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    f = np.empty(sites.shape[0], np.float64)
    fd = np.empty(sites.shape[0], np.float64)
    _check(load_library().ce_read_sites(sim, int(field), sites.shape[0],
                                        sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        _dptr(f), _dptr(fd)), "ce_read_sites")
    return f, fd


def ce_get_step(sim: int) -> int:
    out = ctypes.c_int64()
    _check(load_library().ce_get_step(sim, ctypes.byref(out)), "ce_get_step")
    return out.value


def ce_set_step_block(sim: int, k: int) -> None:
    _check(load_library().ce_set_step_block(sim, int(k)), "ce_set_step_block")


def ce_get_launch(sim: int) -> ce_launch:
    out = ce_launch()
    _check(load_library().ce_get_launch(sim, ctypes.byref(out)), "ce_get_launch")
    return out


def ce_set_launch(sim: int, kernel: int, sites_per_thread: int = 0, lanes_per_row: int = 0,
                  block: int = 0, planes: int = 0, grid: int = 0) -> None:
    cfg = ce_launch(kernel, sites_per_thread, lanes_per_row, block, planes, grid)
    _check(load_library().ce_set_launch(sim, ctypes.byref(cfg)), "ce_set_launch")


def ce_time_steps(sim: int, nsteps: int) -> float:
    ms = ctypes.c_float()
    _check(load_library().ce_time_steps(sim, int(nsteps), ctypes.byref(ms)), "ce_time_steps")
    return ms.value


def ce_sync(sim: int) -> None:
    _check(load_library().ce_sync(sim), "ce_sync")


def ce_destroy(sim: Optional[int]) -> None:
    if sim:
        load_library().ce_destroy(sim)


def ce_spectrum_bins(sim: int) -> int:
    out = ctypes.c_int32()
    _check(load_library().ce_spectrum_bins(sim, ctypes.byref(out)), "ce_spectrum_bins")
    return out.value


def ce_spectrum(sim: int, field: int, want_fdot: bool = True):
    """(power_f, power_fdot or None, count) of field `field`, per radial bin."""
    nb = ce_spectrum_bins(sim)
    pf = np.empty(nb, np.float64)
    pd = np.empty(nb, np.float64) if want_fdot else None
    cnt = np.empty(nb, np.float64)
    _check(load_library().ce_spectrum(sim, int(field), _dptr(pf), _dptr(pd), _dptr(cnt)), "ce_spectrum")
    return pf, pd, cnt


def _u8(buf) -> np.ndarray:
    a = np.frombuffer(buf, np.uint8) if not isinstance(buf, np.ndarray) else buf
    if a.dtype != np.uint8 or not a.flags["C_CONTIGUOUS"]:
        raise ValueError("a grid image is a contiguous uint8 buffer")
    return a


def ce_image_bytes(sim: int) -> int:
    out = ctypes.c_size_t()
    _check(load_library().ce_image_bytes(sim, ctypes.byref(out)), "ce_image_bytes")
    return out.value


def ce_save_image(sim: int, out: Optional[np.ndarray] = None) -> np.ndarray:
    """The simulation's grid image as a uint8 array (written into `out` if given)."""
    n = ce_image_bytes(sim)
    buf = np.empty(n, np.uint8) if out is None else _u8(out)
    _check(load_library().ce_save_image(sim, buf.ctypes.data, buf.nbytes), "ce_save_image")
    return buf[:n]


def ce_image_params(buf) -> ce_params:
    a = _u8(buf)
    out = ce_params()
    _check(load_library().ce_image_params(a.ctypes.data, a.nbytes, ctypes.byref(out)), "ce_image_params")
    return out


def ce_restore_image(sim: int, buf) -> None:
    a = _u8(buf)
    _check(load_library().ce_restore_image(sim, a.ctypes.data, a.nbytes), "ce_restore_image")


class Simulation:
    """Owning handle over one ``ce_sim`` (marshalling only)."""

    def __init__(self, dims: int, N: int, nfields: int, L: float, dt: float, **kw):
        self.dims, self.N, self.nfields = dims, N, nfields
        self.params = make_params(dims, N, nfields, L, dt, **kw)
        self.handle = ce_create(self.params)

    @classmethod
    def from_lattice(cls, lat, precision: int = CE_FP32, **kw) -> "Simulation":
        return cls(lat.dims, lat.N, lat.nfields, lat.L, lat.dt, lam=lat.lam, G=lat.G, mu2=lat.mu2,
                   expansion=lat.expansion, kappa=lat.kappa, precision=precision,
                   vacuum=lat.vacuum, terms=getattr(lat, "terms", None), **kw)

    @classmethod
    def from_image(cls, buf, stream: Optional[int] = None) -> "Simulation":
        """A new simulation resumed from a grid image."""
        p = ce_image_params(buf)
        terms = None
        if p.model == CE_MODEL_POLYNOMIAL:
            terms = [(p.terms[t].coef, tuple(p.terms[t].exp)) for t in range(p.nterms)]
        sim = cls(p.dims, p.N, p.nfields, p.L, p.dt, lam=p.lam, G=list(p.G), mu2=list(p.mu2),
                  expansion=bool(p.expansion), kappa=p.kappa, precision=p.precision, stream=stream,
                  vacuum=p.vacuum, terms=terms)
        try:
            sim.restore_image(buf)
        except Exception:
            sim.close()
            raise
        return sim

    def spectrum(self, field: int, want_fdot: bool = True):
        """Radially binned power spectra (power_f, power_fdot, count) of a field."""
        return ce_spectrum(self.handle, field, want_fdot)

    def save_image(self, out: Optional[np.ndarray] = None) -> np.ndarray:
        return ce_save_image(self.handle, out)

    def restore_image(self, buf) -> None:
        ce_restore_image(self.handle, buf)

    def image_bytes(self) -> int:
        return ce_image_bytes(self.handle)

    @property
    def shape(self):
        return (self.N,) * self.dims

    def load(self, phi: np.ndarray, phidot: np.ndarray, first: int = 0) -> None:
        ce_load_fields(self.handle, first, phi, phidot)

    def generate(self, spec: ce_init_spec) -> None:
        """Generate every field on the device (seeded, see ce_init_spec) and start the run."""
        ce_generate_fields(self.handle, spec)

    def step(self, n: int) -> None:
        ce_step(self.handle, n)

    def energies(self, allow_nonfinite: bool = False) -> ce_energy:
        return ce_energies(self.handle, allow_nonfinite)

    def energy_log(self, count: int):
        return ce_energy_log(self.handle, count)

    def read(self, want_f: bool = True, want_fdot: bool = True):
        return ce_read_fields(self.handle, self.nfields, self.shape, want_f, want_fdot)

    def read_sites(self, field: int, sites: np.ndarray):
        return ce_read_sites(self.handle, field, sites)

    def set_step_block(self, k: int) -> None:
        ce_set_step_block(self.handle, k)

    def get_launch(self) -> ce_launch:
        return ce_get_launch(self.handle)

    def set_launch(self, kernel: int, sites_per_thread: int = 0, lanes_per_row: int = 0,
                   block: int = 0, planes: int = 0, grid: int = 0) -> None:
        ce_set_launch(self.handle, kernel, sites_per_thread, lanes_per_row, block, planes, grid)

    def sync(self) -> None:
        ce_sync(self.handle)

    def time_steps(self, n: int) -> float:
        return ce_time_steps(self.handle, n)

    @property
    def step_count(self) -> int:
        return ce_get_step(self.handle)

    def close(self) -> None:
        if self.handle:
            ce_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- pool ----------------------------------------------------------------

def ce_stream_copy(src: int, dst: int, nbytes: int, streams: int = 4, grid: int = 0, reps: int = 5,
                   stream: Optional[int] = None) -> float:
    """Mean ms of a `streams`-part device copy of nbytes (measurement only)."""
    ms = ctypes.c_float()
    _check(load_library().ce_stream_copy(src, dst, int(nbytes), int(streams), int(grid), int(reps), stream,
                                         ctypes.byref(ms)), "ce_stream_copy")
    return ms.value


CE_PROBE_COPY, CE_PROBE_READ, CE_PROBE_WRITE = 0, 1, 2


def ce_stream_probe(kind: int, src: Optional[int], dst: int, nbytes: int, parts: int = 1, unroll: int = 4,
                    nt: int = 2, grid: int = 0, reps: int = 5, stream: Optional[int] = None) -> float:
    """Mean ms of a measurement stream (copy, read-only or write-only) of nbytes."""
    ms = ctypes.c_float()
    _check(load_library().ce_stream_probe(int(kind), src, dst, int(nbytes), int(parts), int(unroll), int(nt),
                                          int(grid), int(reps), stream, ctypes.byref(ms)), "ce_stream_probe")
    return ms.value


def ce_pool_create(budget_bytes: int, stream: Optional[int] = None) -> int:
    h = ctypes.c_void_p()
    _check(load_library().ce_pool_create(int(budget_bytes), stream, ctypes.byref(h)), "ce_pool_create")
    return h.value


def ce_pool_admit(pool: int, params: ce_params, phi: np.ndarray, phidot: np.ndarray,
                  nsteps: int) -> int:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    phidot = np.ascontiguousarray(phidot, dtype=np.float64)
    jid = ctypes.c_int64()
    _check(load_library().ce_pool_admit(pool, ctypes.byref(params), _dptr(phi), _dptr(phidot),
                                        int(nsteps), ctypes.byref(jid)), "ce_pool_admit")
    return jid.value


def ce_pool_admit_with_launch(pool: int, params: ce_params, launch: Sequence[int], phi: np.ndarray,
                              phidot: np.ndarray, nsteps: int) -> int:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    phidot = np.ascontiguousarray(phidot, dtype=np.float64)
    cfg = ce_launch(*launch)
    jid = ctypes.c_int64()
    _check(load_library().ce_pool_admit_with_launch(pool, ctypes.byref(params), ctypes.byref(cfg), _dptr(phi),
                                                    _dptr(phidot), int(nsteps), ctypes.byref(jid)),
           "ce_pool_admit_with_launch")
    return jid.value


def ce_pool_admit_generated(pool: int, params: ce_params, spec: ce_init_spec, nsteps: int,
                            launch: Optional[Sequence[int]] = None) -> int:
    cfg = ce_launch(*launch) if launch is not None else None
    jid = ctypes.c_int64()
    _check(load_library().ce_pool_admit_generated(pool, ctypes.byref(params),
                                                  ctypes.byref(cfg) if cfg is not None else None,
                                                  ctypes.byref(spec), int(nsteps), ctypes.byref(jid)),
           "ce_pool_admit_generated")
    return jid.value


def ce_pool_launch_for(params: ce_params) -> ce_launch:
    out = ce_launch()
    _check(load_library().ce_pool_launch_for(ctypes.byref(params), ctypes.byref(out)), "ce_pool_launch_for")
    return out


def ce_pool_set_member_launch(pool: int, job_id: int, kernel: int, sites_per_thread: int = 0,
                              lanes_per_row: int = 0, block: int = 0, planes: int = 0,
                              grid: int = 0) -> None:
    cfg = ce_launch(kernel, sites_per_thread, lanes_per_row, block, planes, grid)
    _check(load_library().ce_pool_set_member_launch(pool, int(job_id), ctypes.byref(cfg)),
           "ce_pool_set_member_launch")


def ce_pool_run_block(pool: int, k: int) -> None:
    _check(load_library().ce_pool_run_block(pool, int(k)), "ce_pool_run_block")


def ce_pool_poll(pool: int, job_id: int, want_energy: bool = True, allow_nonfinite: bool = False):
    done = ctypes.c_int32()
    e = ce_energy() if want_energy else None
    allow = (CE_ENONFINITE,) if allow_nonfinite else ()
    _check(load_library().ce_pool_poll(pool, int(job_id), ctypes.byref(done),
                                       ctypes.byref(e) if e is not None else None),
           "ce_pool_poll", allow)
    return bool(done.value), e


def ce_pool_set_quota(pool: int, job_id: int, steps_per_block: int) -> None:
    _check(load_library().ce_pool_set_quota(pool, int(job_id), int(steps_per_block)), "ce_pool_set_quota")


def ce_pool_steps_left(pool: int, job_id: int) -> int:
    left = ctypes.c_int64()
    _check(load_library().ce_pool_steps_left(pool, int(job_id), ctypes.byref(left)), "ce_pool_steps_left")
    return int(left.value)


def ce_pool_retire(pool: int, job_id: int, shape=None, nfields: int = 0):
    f = fd = None
    if shape is not None:
        f = np.empty((nfields,) + tuple(shape), np.float64)
        fd = np.empty((nfields,) + tuple(shape), np.float64)
    _check(load_library().ce_pool_retire(pool, int(job_id), _dptr(f), _dptr(fd)), "ce_pool_retire")
    return f, fd


def ce_pool_save_member(pool: int, job_id: int) -> np.ndarray:
    """Grid image of a pool member (uint8 array); the member stays in the pool."""
    n = ctypes.c_size_t()
    _check(load_library().ce_pool_member_image_bytes(pool, int(job_id), ctypes.byref(n)),
           "ce_pool_member_image_bytes")
    buf = np.empty(n.value, np.uint8)
    _check(load_library().ce_pool_save_member(pool, int(job_id), buf.ctypes.data, buf.nbytes),
           "ce_pool_save_member")
    return buf


def ce_pool_admit_image(pool: int, image, nsteps: int) -> int:
    a = _u8(image)
    jid = ctypes.c_int64()
    _check(load_library().ce_pool_admit_image(pool, a.ctypes.data, a.nbytes, int(nsteps), ctypes.byref(jid)),
           "ce_pool_admit_image")
    return jid.value


def ce_pool_get_info(pool: int) -> ce_pool_info:
    out = ce_pool_info()
    _check(load_library().ce_pool_get_info(pool, ctypes.byref(out)), "ce_pool_get_info")
    return out


def ce_pool_destroy(pool: Optional[int]) -> None:
    if pool:
        load_library().ce_pool_destroy(pool)


class Pool:
    """Owning handle over one ``ce_pool`` (marshalling only)."""

    def __init__(self, budget_bytes: int, stream: Optional[int] = None):
        self.handle = ce_pool_create(budget_bytes, stream)
        self.shapes = {}

    def admit(self, params: ce_params, phi: np.ndarray, phidot: np.ndarray, nsteps: int,
              launch: Optional[Sequence[int]] = None) -> int:
        """Admit a member (launch: optional member launch tuple).  May run on
        another thread than the pool's other calls."""
        if launch is None:
            jid = ce_pool_admit(self.handle, params, phi, phidot, nsteps)
        else:
            jid = ce_pool_admit_with_launch(self.handle, params, launch, phi, phidot, nsteps)
        self.shapes[jid] = ((params.N,) * params.dims, params.nfields)
        return jid

    def admit_generated(self, params: ce_params, spec: ce_init_spec, nsteps: int,
                        launch: Optional[Sequence[int]] = None) -> int:
        """Admit a member whose fields are generated on the device from `spec`."""
        jid = ce_pool_admit_generated(self.handle, params, spec, nsteps, launch)
        self.shapes[jid] = ((params.N,) * params.dims, params.nfields)
        return jid

    def save_member(self, job_id: int) -> np.ndarray:
        """Grid image of a member after its enqueued steps (it stays in the pool)."""
        return ce_pool_save_member(self.handle, job_id)

    def admit_image(self, image, nsteps: int) -> int:
        """Admit a member resumed from a grid image, with nsteps more steps."""
        jid = ce_pool_admit_image(self.handle, image, nsteps)
        p = ce_image_params(image)
        self.shapes[jid] = ((p.N,) * p.dims, p.nfields)
        return jid

    def set_member_launch(self, job_id: int, *cfg) -> None:
        ce_pool_set_member_launch(self.handle, job_id, *cfg)

    def run_block(self, k: int) -> None:
        ce_pool_run_block(self.handle, k)

    def poll(self, job_id: int, want_energy: bool = True, allow_nonfinite: bool = False):
        return ce_pool_poll(self.handle, job_id, want_energy, allow_nonfinite)

    def set_quota(self, job_id: int, steps_per_block: int) -> None:
        """At most this many steps per block for the member (negative: no limit)."""
        ce_pool_set_quota(self.handle, job_id, steps_per_block)

    def steps_left(self, job_id: int) -> int:
        """Steps of the member not yet enqueued (no waiting)."""
        return ce_pool_steps_left(self.handle, job_id)

    def retire(self, job_id: int, read: bool = True):
        shape, nf = self.shapes.pop(job_id)
        return ce_pool_retire(self.handle, job_id, shape if read else None, nf)

    def info(self) -> ce_pool_info:
        return ce_pool_get_info(self.handle)

    def close(self) -> None:
        if self.handle:
            ce_pool_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
