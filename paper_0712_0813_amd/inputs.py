"""Seeded synthetic initial conditions for lattice runs.

This module draws inputs only: it holds none of the evolution's arithmetic and
is shared, as a plain input generator, by the GPU tests, the benchmark and the
CPU oracle's callers.

Recipe (each array independently reproducible from ``(seed, field, kind)``):

* a Gaussian random field on the periodic N^d grid, built in Fourier space from
  every integer wave vector n with 0 < |n| <= N/4 (|n| the Euclidean norm of
  the integer vector, k = 2 pi |n| / L);
* each mode gets a complex amplitude c_n = sigma_n (X + iY), X, Y standard
  normal (Rayleigh modulus, uniform phase), and the real-space field is
  delta(x) = Re sum_n c_n exp(2 pi i n.x / N);
* sigma_n = amp / sqrt(2 omega_k L^d) for a field and
  amp * sqrt(omega_k / 2) / sqrt(L^d) for its time derivative, with
  omega_k = sqrt(k^2 + m_eff^2), m_eff^2 the field's effective mass squared
  at the homogeneous background (passed in by the caller);
* the homogeneous background value is added to the field (the inflaton starts
  at 1, the other fields and all derivatives at 0).

Draws come from ``numpy.random.default_rng(SeedSequence([seed, 2*i + kind]))``
with kind 0 for field i and 1 for its derivative; X then Y are drawn over the
(2K+1)^d box of wave vectors with K = N/4, in C order, so every array can be
generated alone, in any order or in parallel.  The inverse transform runs one
axis at a time over the band-limited box only (zero padding is implicit), with
``scipy.fft`` on all host cores.
"""
from __future__ import annotations

import os
from typing import Sequence, Tuple

import numpy as np
import scipy.fft as sfft

FIELD, MOMENTUM = 0, 1


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def mode_box(dims: int, N: int) -> Tuple[np.ndarray, int]:
    """Integer |n|^2 on the (2K+1)^dims box of wave vectors, K = N//4."""
    K = N // 4
    r = np.arange(-K, K + 1, dtype=np.int64)
    n2 = np.zeros((2 * K + 1,) * dims, np.int64)
    for d in range(dims):
        shape = [1] * dims
        shape[d] = 2 * K + 1
        n2 = n2 + (r * r).reshape(shape)
    return n2, K


def random_field(seed: int, field: int, kind: int, dims: int, N: int, L: float,
                 m_eff2: float, amp: float = 1e-3, workers: int = 0) -> np.ndarray:
    """One fluctuation array delta(x) (float64, shape (N,)*dims), zero mean.
    workers: FFT threads (0: all host cores, up to 16)."""
    if N % 4 != 0 or N < 4:
        raise ValueError("N must be a positive multiple of 4")
    n2, K = mode_box(dims, N)
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 2 * int(field) + int(kind)]))
    X = rng.standard_normal(n2.shape)
    Y = rng.standard_normal(n2.shape)
    k = (2.0 * np.pi / L) * np.sqrt(n2.astype(np.float64))
    omega = np.sqrt(k * k + float(m_eff2))
    inside = (n2 > 0) & (n2 <= K * K)
    with np.errstate(divide="ignore", invalid="ignore"):
        if kind == FIELD:
            sigma = amp / np.sqrt(2.0 * omega * L ** dims)
        else:
            sigma = amp * np.sqrt(omega / 2.0) / np.sqrt(L ** dims)
    sigma = np.where(inside, sigma, 0.0)
    c = sigma * (X + 1j * Y)
    del X, Y, k, omega
    # Hermitian part: Re sum_n c_n e^{i n x} = sum_n H_n e^{i n x},
    # H_n = (c_n + conj(c_{-n})) / 2; keep the half with n_last >= 0.
    flipped = c[(slice(None, None, -1),) * dims]
    H = 0.5 * (c[..., K:] + np.conj(flipped[..., K:]))
    del c, flipped
    # inverse transform axis by axis: sum over modes without the 1/N factor
    w = workers if workers > 0 else _workers()
    for d in range(dims - 1):
        shape = list(H.shape)
        shape[d] = N
        P = np.zeros(shape, np.complex128)
        src_pos = [slice(None)] * dims
        dst_pos = [slice(None)] * dims
        src_pos[d] = slice(K, 2 * K + 1)
        dst_pos[d] = slice(0, K + 1)
        P[tuple(dst_pos)] = H[tuple(src_pos)]
        src_pos[d] = slice(0, K)
        dst_pos[d] = slice(N - K, N)
        P[tuple(dst_pos)] = H[tuple(src_pos)]
        del H
        H = sfft.ifft(P, axis=d, norm="forward", workers=w)
        del P
    out = sfft.irfft(H, n=N, axis=dims - 1, norm="forward", workers=w)
    return np.ascontiguousarray(out, dtype=np.float64)


def make_initial(seed: int, dims: int, N: int, L: float, nfields: int,
                 m_eff2: Sequence[float], amp: float = 1e-3,
                 background: Sequence[float] = (1.0, 0.0, 0.0), workers: int = 0):
    """(phi, phidot), each float64 [nfields, N, ..., N]."""
    shape = (nfields,) + (N,) * dims
    phi = np.empty(shape, np.float64)
    phidot = np.empty(shape, np.float64)
    for i in range(nfields):
        phi[i] = random_field(seed, i, FIELD, dims, N, L, m_eff2[i], amp, workers)
        phi[i] += background[i] if i < len(background) else 0.0
        phidot[i] = random_field(seed, i, MOMENTUM, dims, N, L, m_eff2[i], amp, workers)
    return phi, phidot


def lattice_initial(lat, workers: int = 0):
    """(phi, phidot) for a workloads.Lattice."""
    return make_initial(lat.seed, lat.dims, lat.N, lat.L, lat.nfields, lat.m_eff2(), lat.amp,
                        lat.background, workers)
