"""Synthetic preheating-shaped workloads (program units, lambda = 1).

Every lattice is the two-or-more-field quartic model
V = lambda/4 phi^4 + sum_j G_j/2 phi^2 chi_j^2 (G_j = g_j^2/lambda), started
from phi = 1 plus small Gaussian-random-field fluctuations, chi_j pure
fluctuations (see ``inputs``).  These are the shapes and parameter ranges of
parametric-resonance preheating runs; nothing here is a dataset.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Sequence

import numpy as np

# kappa = 8 pi (phi_0 / M_p)^2 with phi_0 = 0.342 M_p, the inflaton amplitude at
# the end of lambda phi^4 inflation commonly used for preheating studies.
DEFAULT_KAPPA = 8.0 * np.pi * 0.342 ** 2


@dataclass
class Lattice:
    """One lattice run: model, grid, integrator and seed."""
    name: str
    dims: int
    N: int
    nfields: int
    L: float
    dt: float
    steps: int
    G: Sequence[float] = (0.0, 0.0, 0.0)
    mu2: Sequence[float] = (0.0, 0.0, 0.0)
    lam: float = 1.0
    expansion: bool = False
    kappa: float = DEFAULT_KAPPA
    seed: int = 0
    amp: float = 1e-3
    background: Sequence[float] = (1.0, 0.0, 0.0)
    vacuum: float = 0.0     # V0: constant term of the potential (tachyonic / hybrid models)

    @property
    def nsites(self) -> int:
        return self.N ** self.dims

    @property
    def site_fields(self) -> int:
        return self.nsites * self.nfields

    @property
    def dx(self) -> float:
        return self.L / self.N

    def m_eff2(self) -> List[float]:
        """Effective mass^2 of each field at the homogeneous background
        (only used to shape the initial fluctuation spectrum)."""
        b0 = self.background[0]
        out = [3.0 * self.lam * b0 * b0 + self.mu2[0]]
        for j in range(1, self.nfields):
            out.append(self.G[j] * b0 * b0 + self.mu2[j])
        return out

    def with_(self, **kw) -> "Lattice":
        return replace(self, **kw)


# 32^3, static, the small parity case
LATTICE32_STATIC = Lattice("lattice32_static", dims=3, N=32, nfields=2, L=10.0, dt=0.01,
                           steps=200, G=(0.0, 100.0, 0.0), expansion=False, seed=0)
# 256^3 with self-consistent expansion
LATTICE256_EXPANDING = Lattice("lattice256_expanding", dims=3, N=256, nfields=2, L=20.0,
                               dt=0.005, steps=2000, G=(0.0, 100.0, 0.0), expansion=True,
                               seed=0)
# 1024^3 with expansion: the single-GPU throughput / roofline workload
LATTICE1024_EXPANDING = Lattice("lattice1024_expanding", dims=3, N=1024, nfields=2, L=40.0,
                                dt=0.005, steps=500, G=(0.0, 1000.0, 0.0), expansion=True,
                                seed=1)


def ensemble_512x64(count: int = 512, steps: int = 1000) -> List[Lattice]:
    """512 independent 64^3 two-field lattices, seeds 0..count-1, G log-uniform
    in [1, 1e4] (drawn from default_rng(3)), expansion on every odd member."""
    u = np.random.default_rng(3).random(512)
    out = []
    for j in range(count):
        out.append(Lattice(f"ens64_{j}", dims=3, N=64, nfields=2, L=10.0, dt=0.01, steps=steps,
                           G=(0.0, float(10.0 ** (4.0 * u[j])), 0.0),
                           expansion=bool(j % 2), seed=j))
    return out


@dataclass
class Job:
    job_id: int
    arrival: float      # seconds after the stream starts
    lattice: Lattice


def serving_mix(njobs: int = 2000, rate: float = 20.0) -> List[Job]:
    """Poisson stream of mixed jobs: 75% 3-D with N in {32,64,128,256}, 25% 2-D
    with N in {256,512,1024,2048}; 1-3 fields; G_j log-uniform in [1, 1e4];
    steps uniform in 200..2000; expansion for half.  dx = 10/64 and dt = 0.01
    for all jobs; the init seed of job i is 100000 + i."""
    rng = np.random.default_rng(4)
    gaps = rng.exponential(1.0 / rate, njobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for i in range(njobs):
        if rng.random() < 0.75:
            dims, N = 3, int(rng.choice([32, 64, 128, 256]))
        else:
            dims, N = 2, int(rng.choice([256, 512, 1024, 2048]))
        nf = int(rng.integers(1, 4))
        G = [0.0] + [float(10.0 ** (4.0 * rng.random())) for _ in range(nf - 1)]
        G = G + [0.0] * (3 - len(G))
        steps = int(rng.integers(200, 2001))
        expansion = bool(rng.random() < 0.5)
        lat = Lattice(f"job{i}", dims=dims, N=N, nfields=nf, L=N * 10.0 / 64.0, dt=0.01,
                      steps=steps, G=tuple(G), expansion=expansion, seed=100000 + i)
        jobs.append(Job(i, float(arrivals[i]), lat))
    return jobs
