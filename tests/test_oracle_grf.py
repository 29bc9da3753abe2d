"""Pins of the oracle's seeded Gaussian random fields (``oracle/grf.c``)
against things other than itself: NumPy's own Philox4x64-10 bit generator,
the normal distribution, a brute-force count of the wave-vector band, the
direct sum against an FFT, Parseval's identity, and the closed-form variance
of the spectrum."""
import numpy as np
import pytest
from scipy import stats

import oracle

M64 = 2 ** 64 - 1


def numpy_philox_block(counter, key):
    """NumPy's Philox (4x64, 10 rounds) increments its 256-bit counter before
    each block: the block for `counter` comes from a generator set one below."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(counter))
    v = (v - 1) % (1 << 256)
    prev = np.array([(v >> (64 * i)) & M64 for i in range(4)], np.uint64)
    bg = np.random.Philox(counter=prev, key=np.array(key, np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((12345, 3, 0, 0), (7, 0)),
    ((2 ** 63 + 5, 2 ** 40, 17, 2 ** 64 - 1), (2 ** 64 - 1, 99)),
    ((0, 1, 0, 0), (2 ** 32 + 1, 2 ** 63)),
])
def test_philox_matches_numpy(counter, key):
    assert oracle.philox4x64_10(counter, key) == numpy_philox_block(counter, key)


def test_normals_are_standard_normal_and_independent():
    n = 40000
    xy = np.array([oracle.grf_normals(5, b, 3) for b in range(n)])
    X, Y = xy[:, 0], xy[:, 1]
    for v in (X, Y):
        assert abs(v.mean()) < 5 / np.sqrt(n)
        assert abs(v.var() - 1.0) < 5 * np.sqrt(2.0 / n)
        assert stats.kstest(v, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(X, Y)[0, 1]) < 5 / np.sqrt(n)
    # the radius is Rayleigh, the phase uniform
    assert stats.kstest(np.hypot(X, Y), "rayleigh").pvalue > 1e-4
    assert stats.kstest((np.arctan2(Y, X) + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-4
    # different streams and seeds give different numbers
    assert oracle.grf_normals(5, 10, 3) != oracle.grf_normals(5, 10, 2)
    assert oracle.grf_normals(5, 10, 3) != oracle.grf_normals(6, 10, 3)


@pytest.mark.parametrize("dims,N", [(1, 64), (2, 32), (3, 16)])
def test_band_matches_brute_force(dims, N):
    K = N // 4
    c = oracle.grf_modes(1, 0, 0, dims, N, 10.0, 1e-3, 3.0)
    count = 0
    import itertools
    for n in itertools.product(range(-K, K + 1), repeat=dims):
        n2 = sum(v * v for v in n)
        idx = tuple(v + K for v in n)
        inside = 0 < n2 <= K * K
        count += inside
        assert (c[idx] != 0) == inside, n
    assert np.count_nonzero(c) == count


@pytest.mark.parametrize("dims,N,kind", [(1, 32, 0), (2, 16, 1), (3, 8, 0), (3, 12, 1)])
def test_fft_route_equals_direct_sum(dims, N, kind):
    L = 7.0
    delta = oracle.grf_field(3, 1, kind, dims, N, L, 1e-3, 2.0)
    re, im = oracle.grf_mode_parts(3, 1, kind, dims, N, L, 1e-3, 2.0)
    sites = np.arange(N ** dims)
    direct = oracle.grf_sites(re, im, N, sites).reshape((N,) * dims)
    # and a plain Python sum for a few sites, written out from the definition
    K = N // 4
    c = re + 1j * im
    import itertools
    for s in (0, 1, N ** dims // 3, N ** dims - 1):
        x = np.unravel_index(s, (N,) * dims)
        acc = 0.0
        for n in itertools.product(range(-K, K + 1), repeat=dims):
            acc += (c[tuple(v + K for v in n)] * np.exp(2j * np.pi * np.dot(n, x) / N)).real
        assert abs(acc - direct.flat[s]) <= 1e-12 * np.sqrt(np.mean(direct ** 2))
    rms = np.sqrt(np.mean(delta ** 2))
    assert rms > 0
    assert np.max(np.abs(delta - direct)) <= 1e-13 * rms


@pytest.mark.parametrize("dims,N", [(2, 64), (3, 16)])
def test_parseval_and_zero_mean(dims, N):
    K = N // 4
    c = oracle.grf_modes(9, 0, 0, dims, N, 5.0, 1e-3, 3.0)
    delta = oracle.grf_field(9, 0, 0, dims, N, 5.0, 1e-3, 3.0)
    H = 0.5 * (c + np.conj(c[(slice(None, None, -1),) * dims]))
    assert np.isclose(np.mean(delta ** 2), np.sum(np.abs(H) ** 2), rtol=1e-12)
    assert abs(np.mean(delta)) <= 1e-14 * np.sqrt(np.mean(delta ** 2))


@pytest.mark.parametrize("kind", [0, 1])
def test_variance_matches_spectrum(kind):
    # E[delta(x)^2] = sum_n sigma_n^2 over the band (each mode contributes
    # Var Re(c_n e^{i theta}) = sigma_n^2); averaged over sites and seeds
    dims, N, L, amp, m2 = 3, 16, 6.0, 1e-3, 3.0
    K = N // 4
    r = np.arange(-K, K + 1)
    n2 = sum(np.meshgrid(*([r * r] * dims), indexing="ij"))
    band = (n2 > 0) & (n2 <= K * K)
    k = 2 * np.pi * np.sqrt(n2[band]) / L
    w = np.sqrt(k * k + m2)
    sig2 = amp ** 2 / (2 * w * L ** dims) if kind == 0 else amp ** 2 * (w / 2) / L ** dims
    expect = np.sum(sig2)
    got = np.mean([np.mean(oracle.grf_field(s, 0, kind, dims, N, L, amp, m2) ** 2) for s in range(24)])
    assert abs(got / expect - 1.0) < 0.06
