"""The synthetic workloads carry the sizes and physics they are named for,
and every lattice among them is leapfrog-stable at its couplings."""
import numpy as np

from paper_0712_0813_amd import ce
from paper_0712_0813_amd.workloads import (LATTICE32_STATIC, LATTICE256_EXPANDING, LATTICE1024_EXPANDING,
                                           ensemble_512x64)


def _stable(lat):
    # dt sqrt(4 d / dx^2 + largest curvature at the background) < 2
    m2 = max(lat.m_eff2())
    return lat.dt * np.sqrt(4 * lat.dims / lat.dx ** 2 + m2) < 2


def test_single_lattices():
    for lat, want in [
        (LATTICE32_STATIC, dict(dims=3, N=32, nfields=2, L=10.0, dt=0.01, steps=200, G1=100.0, expansion=False, seed=0)),
        (LATTICE256_EXPANDING, dict(dims=3, N=256, nfields=2, L=20.0, dt=0.005, steps=2000, G1=100.0,
                                    expansion=True, seed=0)),
        (LATTICE1024_EXPANDING, dict(dims=3, N=1024, nfields=2, L=40.0, dt=0.005, steps=500, G1=1000.0,
                                     expansion=True, seed=1)),
    ]:
        got = dict(dims=lat.dims, N=lat.N, nfields=lat.nfields, L=lat.L, dt=lat.dt, steps=lat.steps, G1=lat.G[1],
                   expansion=lat.expansion, seed=lat.seed)
        assert got == want, lat.name
        assert lat.lam == 1.0 and tuple(lat.background[:2]) == (1.0, 0.0)
        assert _stable(lat)
        # the library accepts it (validation only, no device work)
        p = ce.make_params(lat.dims, lat.N, lat.nfields, lat.L, lat.dt, G=lat.G, expansion=lat.expansion,
                           kappa=lat.kappa)
        assert ce.ce_required_bytes(p) > 0


def test_ensemble_512x64():
    ens = ensemble_512x64()
    assert len(ens) == 512
    assert {(l.dims, l.N, l.nfields, l.L, l.dt, l.steps) for l in ens} == {(3, 64, 2, 10.0, 0.01, 1000)}
    assert [l.seed for l in ens] == list(range(512))
    assert sum(l.expansion for l in ens) == 256 and all(l.expansion == bool(j % 2) for j, l in enumerate(ens))
    G = np.array([l.G[1] for l in ens])
    assert G.min() >= 1.0 and G.max() <= 1e4
    # log-uniform: the decades are about equally filled
    counts = np.histogram(np.log10(G), bins=4, range=(0, 4))[0]
    assert counts.min() > 90
    assert all(_stable(l) for l in ens)
    # a shorter ensemble is a prefix of the same members
    assert [l.G for l in ensemble_512x64(count=8)] == [l.G for l in ens[:8]]
