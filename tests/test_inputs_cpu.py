"""The seeded host input generator shared by the tests and the benchmark
(paper_0712_0813_amd/inputs.py): determinism, the band of wave vectors, zero
mean, and agreement with the direct sum Re sum_n c_n exp(2 pi i n.x/N) over
the same draws."""
import itertools

import numpy as np
import pytest

from paper_0712_0813_amd.inputs import FIELD, MOMENTUM, make_initial, mode_box, random_field


def test_deterministic_and_independent_streams():
    a = random_field(3, 0, FIELD, 3, 16, 5.0, 3.0)
    assert np.array_equal(a, random_field(3, 0, FIELD, 3, 16, 5.0, 3.0))
    assert np.array_equal(a, random_field(3, 0, FIELD, 3, 16, 5.0, 3.0, workers=1))
    for other in (random_field(4, 0, FIELD, 3, 16, 5.0, 3.0), random_field(3, 1, FIELD, 3, 16, 5.0, 3.0),
                  random_field(3, 0, MOMENTUM, 3, 16, 5.0, 3.0)):
        assert not np.allclose(a, other)


@pytest.mark.parametrize("dims,N", [(1, 64), (2, 16), (3, 8)])
def test_band_and_zero_mean(dims, N):
    d = random_field(11, 0, FIELD, dims, N, 4.0, 1.0)
    F = np.fft.fftn(d)
    K = N // 4
    n = np.fft.fftfreq(N, 1.0 / N).astype(np.int64)
    n2 = sum(np.meshgrid(*([n * n] * dims), indexing="ij"))
    band = (n2 > 0) & (n2 <= K * K)
    scale = np.max(np.abs(F))
    assert scale > 0
    assert np.max(np.abs(F[~band])) <= 1e-12 * scale
    assert abs(d.mean()) <= 1e-14 * np.sqrt(np.mean(d * d))


def test_equals_direct_sum_over_the_same_draws():
    # redraw c_n = sigma_n (X + iY) exactly as documented and sum
    # Re c_n e^{2 pi i n.x/N} site by site
    seed, field, kind, dims, N, L, m2, amp = 5, 1, MOMENTUM, 2, 8, 3.0, 2.0, 1e-3
    got = random_field(seed, field, kind, dims, N, L, m2, amp)
    n2, K = mode_box(dims, N)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2 * field + kind]))
    X = rng.standard_normal(n2.shape)
    Y = rng.standard_normal(n2.shape)
    want = np.zeros((N,) * dims)
    for idx in itertools.product(range(2 * K + 1), repeat=dims):
        nv = np.array(idx) - K
        q = int(nv @ nv)
        if q == 0 or q > K * K:
            continue
        k = 2.0 * np.pi / L * np.sqrt(q)
        omega = np.sqrt(k * k + m2)
        sigma = amp * np.sqrt(omega / 2.0) / np.sqrt(L ** dims)
        c = sigma * (X[idx] + 1j * Y[idx])
        for x in itertools.product(range(N), repeat=dims):
            want[x] += (c * np.exp(2j * np.pi * (nv @ np.array(x)) / N)).real
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_make_initial_backgrounds():
    phi, phid = make_initial(2, 3, 8, 2.5, 2, [3.0, 100.0], amp=1e-3, background=(1.0, 0.0, 0.0))
    assert phi.shape == phid.shape == (2, 8, 8, 8)
    assert abs(phi[0].mean() - 1.0) < 1e-12 and abs(phi[1].mean()) < 1e-12
    assert abs(phid.mean()) < 1e-12
    assert 0 < np.std(phi[0]) < 1e-2
