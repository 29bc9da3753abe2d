"""The largest jobs of the serving stream at their own size, as pool members
with the pool's default member launches (the ones the server uses without a
tuning cache): a 256^3 and a 2048^2 lattice, three fields each, expanding,
in one pool at once.

The oracle cannot evolve them here, so each input is a seeded 32^3 (256^2)
field tiled periodically to the full size: a periodic lattice made of
identical tiles evolves exactly like one tile, so the oracle's run of one
tile fixes every site.  After 100 steps in pool blocks, sampled sites and the
final diagnostics are compared with the oracle, and images of a site in
different tiles must agree bitwise.
"""
import numpy as np
import pytest

from paper_0712_0813_amd import ce
from oracle import Oracle
from _parity import TOL_MEAN, TOL_SITE, Case, energy_errors

pytestmark = pytest.mark.gpu

STEPS = 100
# (full N, tile case); dx = 10/64 and dt = 0.01 as in the serving stream
JOBS = [
    (256, Case("serve_cube_3f", 3, 32, 3, 32 * 10.0 / 64, 0.01, G=(0.0, 50.0, 2000.0), expansion=True, seed=61)),
    (2048, Case("serve_square_3f", 2, 256, 3, 256 * 10.0 / 64, 0.01, G=(0.0, 300.0, 8000.0), expansion=True,
                seed=62)),
]


def _full_params(case, N):
    return ce.make_params(case.dims, N, case.nfields, case.L * N / case.N, case.dt, lam=case.lam, G=case.G,
                          mu2=case.mu2, expansion=case.expansion, kappa=case.kappa)


def test_largest_serving_jobs_in_one_pool_against_oracle():
    orcs, ids, tiles = [], [], []
    with ce.Pool(16 << 30) as pool:
        for N, case in JOBS:
            phi, phid = case.inputs()
            reps = (1,) + (N // case.N,) * case.dims
            print(f"[serve-full] admit {case.name} N={N}", flush=True)
            ids.append(pool.admit(_full_params(case, N), np.tile(phi, reps), np.tile(phid, reps), STEPS))
            orcs.append(Oracle(case.oracle_params(), phi, phid))
        assert pool.info().active == 2
        while pool.info().active > 0:
            pool.run_block(16)
        for o in orcs:
            o.step(STEPS)
        rng = np.random.default_rng(5)
        for (N, case), jid, o in zip(JOBS, ids, orcs):
            done, e = pool.poll(jid)
            assert done and e.step == STEPS
            errs = energy_errors(e.as_dict(case.nfields), o.log[-1], case.nfields)
            worst = max(errs, key=errs.get)
            assert errs[worst] <= TOL_MEAN[ce.CE_FP32], (case.name, worst, errs[worst])
            f, fd = pool.retire(jid, read=True)
            shape = (N,) * case.dims
            sites = rng.integers(0, N ** case.dims, 50000)
            idx = np.unravel_index(sites, shape)
            base = np.ravel_multi_index(tuple(x % case.N for x in idx), (case.N,) * case.dims)
            # the same tile site, some tiles away along every axis
            shifted = np.ravel_multi_index(tuple((x + case.N * (3 + 2 * k)) % N for k, x in enumerate(idx)), shape)
            for i in range(case.nfields):
                for got, want in ((f[i].ravel(), o.f[i].ravel()), (fd[i].ravel(), o.pi[i].ravel())):
                    rms = np.sqrt(np.mean(want * want))
                    err = np.max(np.abs(got[sites] - want[base]) / np.maximum(np.abs(want[base]), rms))
                    assert err <= TOL_SITE[ce.CE_FP32], (case.name, i, err)
                    assert np.array_equal(got[sites], got[shifted]), (case.name, i)
            print(f"[serve-full] {case.name} ok", flush=True)
