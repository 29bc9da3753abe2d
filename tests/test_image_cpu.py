"""Grid-image header handling on the host (no device work): the ctypes
layout of the documented header and ce_image_params' checks."""
import ctypes

import numpy as np
import pytest

from paper_0712_0813_amd import ce


def header(**over):
    h = ce.ce_image_header()
    magic = over.pop("magic", ce.IMAGE_MAGIC)   # written as raw bytes: it holds NULs
    h.version = ce.IMAGE_VERSION
    h.header_bytes = 512
    h.dims, h.N, h.nfields, h.precision, h.model, h.expansion = 3, 16, 2, ce.CE_FP32, 0, 1
    h.L, h.dt, h.lam = 5.0, 0.01, 1.0
    h.G[1] = 100.0
    h.mu2[0] = 0.25
    h.kappa = 2.9
    h.vacuum = 0.25
    h.step = 123
    h.state_bytes = 1024
    h.ring_bytes = ce.ENERGY_LOG * ctypes.sizeof(ce.ce_energy)
    h.field_bytes = 16 ** 3 * 4
    for k, v in over.items():
        setattr(h, k, v)
    if "total_bytes" not in over:
        h.total_bytes = 512 + h.state_bytes + h.ring_bytes + 2 * h.nfields * h.field_bytes
    buf = np.zeros(h.total_bytes, np.uint8)
    buf[:512] = np.frombuffer(bytes(h), np.uint8)
    buf[:8] = np.frombuffer(magic, np.uint8)
    return buf


def test_header_layout():
    assert ctypes.sizeof(ce.ce_image_header) == 512
    off = {n: getattr(ce.ce_image_header, n).offset for n, _ in ce.ce_image_header._fields_}
    assert off["version"] == 8 and off["dims"] == 16 and off["L"] == 40 and off["kappa"] == 112
    assert off["step"] == 120 and off["launch"] == 128 and off["state_bytes"] == 152
    assert off["total_bytes"] == 176 and off["vacuum"] == 184 and off["nterms"] == 192
    assert off["terms"] == 200 and off["reserved"] == 392
    assert ctypes.sizeof(ce.ce_term) == 24


def test_polynomial_params_round_trip():
    terms = (ce.ce_term * ce.MAX_TERMS)()
    terms[0] = ce.ce_term(0.25, (ctypes.c_int32 * 3)(6, 0, 0), 0)
    terms[1] = ce.ce_term(-2.0, (ctypes.c_int32 * 3)(1, 2, 0), 0)
    buf = header(model=ce.CE_MODEL_POLYNOMIAL, lam=0.0, G=(ctypes.c_double * 3)(), mu2=(ctypes.c_double * 3)(),
                 vacuum=0.0, nterms=2, terms=terms)
    p = ce.ce_image_params(buf)
    assert p.model == ce.CE_MODEL_POLYNOMIAL and p.nterms == 2
    assert (p.terms[0].coef, list(p.terms[0].exp)) == (0.25, [6, 0, 0])
    assert (p.terms[1].coef, list(p.terms[1].exp)) == (-2.0, [1, 2, 0])


def test_params_round_trip():
    p = ce.ce_image_params(header())
    assert (p.dims, p.N, p.nfields, p.precision, p.expansion) == (3, 16, 2, ce.CE_FP32, 1)
    assert (p.L, p.dt, p.lam, p.kappa, p.vacuum) == (5.0, 0.01, 1.0, 2.9, 0.25)
    assert list(p.G) == [0.0, 100.0, 0.0] and list(p.mu2) == [0.25, 0.0, 0.0]
    assert p.stream is None and p.arena is None


@pytest.mark.parametrize("what", ["magic", "version", "header_bytes", "field_bytes", "total", "truncated",
                                  "dims", "unstable", "nterms", "terms_with_quartic"])
def test_params_rejections(what):
    if what == "magic":
        buf = header(magic=b"CEGRID\0\2")
    elif what == "version":
        buf = header(version=1)
    elif what == "header_bytes":
        buf = header(header_bytes=128)
    elif what == "field_bytes":
        buf = header(field_bytes=16 ** 3 * 8)
    elif what == "total":
        good = header()
        buf = header(total_bytes=good.nbytes + 4)
    elif what == "truncated":
        buf = header()[:-1].copy()
    elif what == "dims":
        buf = header(dims=4)
    elif what == "nterms":
        buf = header(model=ce.CE_MODEL_POLYNOMIAL, lam=0.0, G=(ctypes.c_double * 3)(), mu2=(ctypes.c_double * 3)(),
                     vacuum=0.0, nterms=9)
    elif what == "terms_with_quartic":
        buf = header(nterms=1)
    else:
        buf = header(dt=0.5)
    with pytest.raises(ce.CeError) as e:
        ce.ce_image_params(buf)
    assert e.value.status == ce.CE_EINVAL
    with pytest.raises(ce.CeError):
        ce.ce_image_params(buf[:100].copy())
