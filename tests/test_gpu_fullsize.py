"""Full-size (1024^3, two fields, FP32, expansion on) parity in the launch
configuration the benchmark times: the tuned launch of the class when the
tuning cache holds one for the current sources, else the library default.

The oracle cannot evolve 1024^3 here, so the input is a seeded 32^3 field
(same dx, dt, couplings and expansion) tiled 32 times along every axis.  A
periodic lattice made of identical tiles evolves exactly like one tile (every
volume mean is the same), so the oracle's 32^3 run fixes every site of the
1024^3 run; sampled sites are compared one by one, and images of a site in
different tiles must agree bitwise.
"""
import numpy as np
import pytest

from paper_0712_0813_amd import autotune, ce
from paper_0712_0813_amd.workloads import LATTICE1024_EXPANDING
from oracle import Oracle
from _parity import TOL_MEAN, TOL_SITE, Case, energy_errors, rounded

pytestmark = pytest.mark.gpu

W = LATTICE1024_EXPANDING
BASE = 32


@pytest.mark.parametrize("precision", [ce.CE_FP32, ce.CE_FP64], ids=["fp32", "fp64"])
def test_full_size_tiled_against_oracle(precision):
    reps = W.N // BASE
    base = Case("tile", 3, BASE, W.nfields, W.L * BASE / W.N, W.dt, G=tuple(W.G), expansion=True,
                kappa=W.kappa, seed=W.seed)
    phi, phid = base.inputs()
    steps = 64
    sites = np.random.default_rng(2).integers(0, W.N ** 3, 100000)
    with ce.Simulation.from_lattice(W, precision=precision) as s:
        tuned = autotune.lookup(W.dims, W.N, W.nfields, precision)
        if tuned:
            s.set_launch(*tuned)
        print(f"[fullsize] 1024^3 launch {s.get_launch().as_tuple()}", flush=True)
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
    orc = Oracle(base.oracle_params(), rounded(phi, precision), rounded(phid, precision))
    orc.step(steps)
    z, y, x = np.unravel_index(sites, (W.N,) * 3)
    bsite = np.ravel_multi_index((z % BASE, y % BASE, x % BASE), (BASE,) * 3)
    for i in range(W.nfields):
        of = orc.f[i].ravel()
        op = orc.pi[i].ravel()
        rms_f, rms_p = np.sqrt(np.mean(of ** 2)), np.sqrt(np.mean(op ** 2))
        ef = np.max(np.abs(got[i][0] - of[bsite]) / np.maximum(np.abs(of[bsite]), rms_f))
        ep = np.max(np.abs(got[i][1] - op[bsite]) / np.maximum(np.abs(op[bsite]), rms_p))
        assert ef <= TOL_SITE[precision], (i, ef)
        assert ep <= TOL_SITE[precision], (i, ep)
        assert np.array_equal(img[i][0], got[i][0][:2000])
        assert np.array_equal(img[i][1], got[i][1][:2000])
    for k, (g, o) in enumerate(zip(log, orc.log)):
        errs = energy_errors(g, o, W.nfields)
        worst = max(errs, key=errs.get)
        assert errs[worst] <= TOL_MEAN[precision], (k, worst, errs[worst])


def test_256_expanding_full_length_tiled_against_oracle():
    # the 256^3 expanding workload at its own size and length (2000 steps,
    # tau = 10): per site after 200 steps, volume averages every 100 steps
    # to the end, and tile images bitwise throughout
    from paper_0712_0813_amd.workloads import LATTICE256_EXPANDING as W2
    reps = W2.N // BASE
    base = Case("tile256", 3, BASE, W2.nfields, W2.L * BASE / W2.N, W2.dt, G=tuple(W2.G), expansion=True,
                kappa=W2.kappa, seed=W2.seed)
    phi, phid = base.inputs()
    orc = Oracle(base.oracle_params(), phi, phid)
    sites = np.random.default_rng(3).integers(0, W2.N ** 3, 20000)
    z, y, x = np.unravel_index(sites, (W2.N,) * 3)
    bsite = np.ravel_multi_index((z % BASE, y % BASE, x % BASE), (BASE,) * 3)
    shifted = np.ravel_multi_index(((z + BASE * 3) % W2.N, (y + BASE * 5) % W2.N, (x + BASE * 6) % W2.N),
                                   (W2.N,) * 3)
    with ce.Simulation.from_lattice(W2, precision=ce.CE_FP32) as s:
        # the launch the benchmark's 256^3 leg runs
        tuned = autotune.lookup(W2.dims, W2.N, W2.nfields, ce.CE_FP32)
        if tuned:
            s.set_launch(*tuned)
        print(f"[fullsize] 256^3 launch {s.get_launch().as_tuple()}", flush=True)
        for i in range(W2.nfields):
            s.load(np.tile(phi[i:i + 1], (1, reps, reps, reps)),
                   np.tile(phid[i:i + 1], (1, reps, reps, reps)), first=i)
        samples = [(s.energies().as_dict(W2.nfields), orc.state)]
        for block in range(W2.steps // 100):
            s.step(100)
            o = orc.step(100, record=False)
            samples.append((s.energies().as_dict(W2.nfields), o))
            if block == 1:   # step 200: per site
                for i in range(W2.nfields):
                    f, fd = s.read_sites(i, sites)
                    of, op = orc.f[i].ravel(), orc.pi[i].ravel()
                    rf, rp = np.sqrt(np.mean(of ** 2)), np.sqrt(np.mean(op ** 2))
                    assert np.max(np.abs(f - of[bsite]) / np.maximum(np.abs(of[bsite]), rf)) <= TOL_SITE[ce.CE_FP32]
                    assert np.max(np.abs(fd - op[bsite]) / np.maximum(np.abs(op[bsite]), rp)) <= TOL_SITE[ce.CE_FP32]
        for i in range(W2.nfields):
            a = s.read_sites(i, sites)
            b = s.read_sites(i, shifted)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for g, o in samples:
        assert g["step"] == o.step
        errs = energy_errors(g, o, W2.nfields)
        worst = max(errs, key=errs.get)
        assert errs[worst] <= 1e-3, (o.step, worst, errs[worst])
