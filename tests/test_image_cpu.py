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
    h.header_bytes = 256
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
        h.total_bytes = 256 + h.state_bytes + h.ring_bytes + 2 * h.nfields * h.field_bytes
    buf = np.zeros(h.total_bytes, np.uint8)
    buf[:256] = np.frombuffer(bytes(h), np.uint8)
    buf[:8] = np.frombuffer(magic, np.uint8)
    return buf


def test_header_layout():
    assert ctypes.sizeof(ce.ce_image_header) == 256
    off = {n: getattr(ce.ce_image_header, n).offset for n, _ in ce.ce_image_header._fields_}
    assert off["version"] == 8 and off["dims"] == 16 and off["L"] == 40 and off["kappa"] == 112
    assert off["step"] == 120 and off["launch"] == 128 and off["state_bytes"] == 152
    assert off["total_bytes"] == 176 and off["vacuum"] == 184 and off["reserved"] == 192


def test_params_round_trip():
    p = ce.ce_image_params(header())
    assert (p.dims, p.N, p.nfields, p.precision, p.expansion) == (3, 16, 2, ce.CE_FP32, 1)
    assert (p.L, p.dt, p.lam, p.kappa, p.vacuum) == (5.0, 0.01, 1.0, 2.9, 0.25)
    assert list(p.G) == [0.0, 100.0, 0.0] and list(p.mu2) == [0.25, 0.0, 0.0]
    assert p.stream is None and p.arena is None


@pytest.mark.parametrize("what", ["magic", "version", "header_bytes", "field_bytes", "total", "truncated",
                                  "dims", "unstable"])
def test_params_rejections(what):
    if what == "magic":
        buf = header(magic=b"CEGRID\0\2")
    elif what == "version":
        buf = header(version=2)
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
    else:
        buf = header(dt=0.5)
    with pytest.raises(ce.CeError) as e:
        ce.ce_image_params(buf)
    assert e.value.status == ce.CE_EINVAL
    with pytest.raises(ce.CeError):
        ce.ce_image_params(buf[:100].copy())
