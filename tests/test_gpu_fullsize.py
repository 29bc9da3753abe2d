"""Full-size (1024^3, two fields, FP32, expansion on) parity in the launch
configuration the benchmark times.

The oracle cannot evolve 1024^3 here, so the input is a seeded 32^3 field
(same dx, dt, couplings and expansion) tiled 32 times along every axis.  A
periodic lattice made of identical tiles evolves exactly like one tile (every
volume mean is the same), so the oracle's 32^3 run fixes every site of the
1024^3 run; sampled sites are compared one by one, and images of a site in
different tiles must agree bitwise.
"""
import numpy as np
import pytest

from paper_0712_0813_amd import ce
from paper_0712_0813_amd.workloads import LATTICE1024_EXPANDING
from oracle import Oracle
from _parity import TOL_MEAN, TOL_SITE, Case, energy_errors, rounded

pytestmark = pytest.mark.gpu

W = LATTICE1024_EXPANDING
BASE = 32


def test_full_size_tiled_against_oracle():
    reps = W.N // BASE
    base = Case("tile", 3, BASE, W.nfields, W.L * BASE / W.N, W.dt, G=tuple(W.G), expansion=True,
                kappa=W.kappa, seed=W.seed)
    phi, phid = base.inputs()
    steps = 64
    sites = np.random.default_rng(2).integers(0, W.N ** 3, 100000)
    with ce.Simulation.from_lattice(W, precision=ce.CE_FP32) as s:
        for i in range(W.nfields):
            s.load(np.tile(phi[i:i + 1], (1, reps, reps, reps)),
                   np.tile(phid[i:i + 1], (1, reps, reps, reps)), first=i)
        s.step(steps)
        got = [s.read_sites(i, sites) for i in range(W.nfields)]
        # images of the same tile site in other tiles
        z, y, x = np.unravel_index(sites[:2000], (W.N,) * 3)
        shifted = np.ravel_multi_index(((z + BASE * 7) % W.N, (y + BASE * 13) % W.N,
                                        (x + BASE * 29) % W.N), (W.N,) * 3)
        img = [s.read_sites(i, shifted) for i in range(W.nfields)]
        log = [e.as_dict(W.nfields) for e in s.energy_log(steps + 1)]
    orc = Oracle(base.oracle_params(), rounded(phi, ce.CE_FP32), rounded(phid, ce.CE_FP32))
    orc.step(steps)
    z, y, x = np.unravel_index(sites, (W.N,) * 3)
    bsite = np.ravel_multi_index((z % BASE, y % BASE, x % BASE), (BASE,) * 3)
    for i in range(W.nfields):
        of = orc.f[i].ravel()
        op = orc.pi[i].ravel()
        rms_f, rms_p = np.sqrt(np.mean(of ** 2)), np.sqrt(np.mean(op ** 2))
        ef = np.max(np.abs(got[i][0] - of[bsite]) / np.maximum(np.abs(of[bsite]), rms_f))
        ep = np.max(np.abs(got[i][1] - op[bsite]) / np.maximum(np.abs(op[bsite]), rms_p))
        assert ef <= TOL_SITE[ce.CE_FP32], (i, ef)
        assert ep <= TOL_SITE[ce.CE_FP32], (i, ep)
        assert np.array_equal(img[i][0], got[i][0][:2000])
        assert np.array_equal(img[i][1], got[i][1][:2000])
    for k, (g, o) in enumerate(zip(log, orc.log)):
        errs = energy_errors(g, o, W.nfields)
        worst = max(errs, key=errs.get)
        assert errs[worst] <= TOL_MEAN[ce.CE_FP32], (k, worst, errs[worst])
