"""Pins of the oracle's radially binned power spectrum against brute force
(explicit DFT sums and mode enumeration), Parseval's identity and closed
forms (a constant, a single cosine)."""
import itertools
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("dims,N", [(1, 16), (2, 8), (3, 4)])
def test_brute_force_dft_and_binning(dims, N):
    g = np.random.default_rng(dims).standard_normal((N,) * dims)
    power, count = oracle.spectrum(g)
    nb = oracle.spectrum_bins(dims, N)
    bp, bc = np.zeros(nb), np.zeros(nb)
    freqs = [v if v < N // 2 else v - N for v in range(N)]
    for n in itertools.product(freqs, repeat=dims):
        F = 0.0
        for x in itertools.product(range(N), repeat=dims):
            F += g[x] * np.exp(-2j * np.pi * np.dot(n, x) / N)
        F /= N ** dims
        j = math.isqrt(sum(v * v for v in n))
        bp[j] += abs(F) ** 2
        bc[j] += 1
    assert np.array_equal(count, bc)
    assert np.allclose(power, bp, rtol=1e-12, atol=1e-15 * bp.sum())


@pytest.mark.parametrize("dims,N", [(2, 64), (3, 16)])
def test_parseval_and_counts(dims, N):
    g = 1.0 + 0.1 * np.random.default_rng(5).standard_normal((N,) * dims)
    power, count = oracle.spectrum(g)
    assert np.isclose(power.sum(), np.mean(g * g), rtol=1e-13)
    assert count.sum() == N ** dims
    assert len(power) == math.isqrt(dims * (N // 2) ** 2) + 1


def test_constant_and_single_mode():
    N = 16
    x = np.indices((N, N, N))
    power, _ = oracle.spectrum(np.full((N, N, N), 3.0))
    assert power[0] == pytest.approx(9.0, rel=1e-15) and np.all(np.abs(power[1:]) < 1e-28)
    m = (1, 2, 0)
    g = 0.5 * np.cos(2 * np.pi * (m[0] * x[0] + m[1] * x[1] + m[2] * x[2]) / N)
    power, _ = oracle.spectrum(g)
    # A cos(k.x) puts A^2/4 at each of n = +m and -m: bin floor(sqrt 5) = 2
    j = math.isqrt(sum(v * v for v in m))
    assert power[j] == pytest.approx(0.5 ** 2 / 2, rel=1e-13)
    assert np.sum(np.delete(power, j)) < 1e-28
