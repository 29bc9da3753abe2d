"""User-defined polynomial potentials on the GPU against the oracle.

Models given as terms of V(phi) = sum_t coef_t prod_i phi_i^e_ti run through
every kernel family (direct 1-D and 3-D, tiled 3-D, streaming 2-D), in FP64
and FP32, with and without expansion; per site after 200 steps and the
volume means every step match the oracle (which evaluates the same
polynomial by its plain definition).  The quartic workload spelled as terms
follows the quartic model's trajectory on the device; polynomial pool
members are bitwise their lone runs; a grid image of a polynomial run
resumes bitwise; a potential too stiff for the time step is refused.
"""
import numpy as np
import pytest

from paper_0712_0813_amd import ce
from oracle import Oracle
from _parity import TOL_MEAN, TOL_SITE, Case, energy_errors, site_error

pytestmark = pytest.mark.gpu

# phi^6 self-interaction and phi^2 chi^2 coupling with masses (degrees 6, 4, 2)
SEXTIC = ((0.25, (4, 0, 0)), (0.02, (6, 0, 0)), (50.0, (2, 2, 0)), (0.1, (2, 0, 0)), (0.3, (0, 2, 0)))
# three fields with a trilinear coupling, a cubic term and a vacuum energy (degrees 4, 3, 2, 0)
TRILINEAR = ((0.25, (4, 0, 0)), (20.0, (2, 2, 0)), (15.0, (2, 0, 2)), (0.5, (1, 1, 1)), (-0.05, (3, 0, 0)),
             (0.2, (0, 2, 0)), (0.05, (0, 0, 0)))
# the double well lambda/4 (phi^2 - v^2)^2 expanded, v = 1, beside chi
DOUBLE_WELL = ((0.25, (4, 0, 0)), (-0.5, (2, 0, 0)), (0.25, (0, 0, 0)), (40.0, (2, 2, 0)))

KAPPA = 2.94
CASES = [
    (Case("sextic3d_direct_exp", 3, 32, 2, 5.0, 0.01, lam=0.0, expansion=True, kappa=KAPPA, seed=81,
          terms=SEXTIC), ce.CE_FP64),
    (Case("sextic3d_direct_exp", 3, 32, 2, 5.0, 0.01, lam=0.0, expansion=True, kappa=KAPPA, seed=81,
          terms=SEXTIC), ce.CE_FP32),
    (Case("sextic3d_tiled", 3, 64, 2, 10.0, 0.01, lam=0.0, expansion=True, kappa=KAPPA, seed=82,
          terms=SEXTIC), ce.CE_FP32),
    (Case("sextic3d_tiled_fp64", 3, 64, 2, 10.0, 0.01, lam=0.0, seed=82, terms=SEXTIC), ce.CE_FP64),
    (Case("trilinear2d_stream", 2, 256, 3, 40.0, 0.01, lam=0.0, expansion=True, kappa=0.5, seed=83,
          terms=TRILINEAR), ce.CE_FP32),
    (Case("trilinear2d_stream_fp64", 2, 256, 3, 40.0, 0.01, lam=0.0, seed=83, terms=TRILINEAR), ce.CE_FP64),
    (Case("doublewell1d", 1, 512, 2, 80.0, 0.02, lam=0.0, expansion=True, kappa=0.05, background=(0.1, 0.0, 0.0),
          seed=84, terms=DOUBLE_WELL), ce.CE_FP64),
]


@pytest.mark.parametrize("case,precision", CASES, ids=[f"{c[0].name}_{'fp64' if c[1] else 'fp32'}" for c in CASES])
def test_polynomial_against_oracle(case, precision):
    steps = 200
    phi, phid = case.inputs()
    orc = Oracle(case.oracle_params(), phi, phid)
    orc.step(steps)
    with case.sim(precision) as s:
        s.load(phi, phid)
        s.step(steps)
        f, fd = s.read()
        log = [e.as_dict(case.nfields) for e in s.energy_log(steps + 1)]
        launch = s.get_launch().as_tuple()
    print(f"[poly] {case.name} launch {launch}", flush=True)
    for i in range(case.nfields):
        assert site_error(f[i], orc.f[i]) <= TOL_SITE[precision], (i, site_error(f[i], orc.f[i]))
        assert site_error(fd[i], orc.pi[i]) <= TOL_SITE[precision], (i, site_error(fd[i], orc.pi[i]))
    for g, o in zip(log, orc.log):
        errs = energy_errors(g, o, case.nfields)
        worst = max(errs, key=errs.get)
        assert errs[worst] <= TOL_MEAN[precision], (g["step"], worst, errs[worst])
        if case.expansion:
            assert abs(g["friedmann_residual"] - o.resid) <= TOL_MEAN[precision]


def _quartic_terms(G, mu2):
    return ((0.25, (4, 0, 0)), (0.5 * G, (2, 2, 0)), (0.5 * mu2[0], (2, 0, 0)), (0.5 * mu2[1], (0, 2, 0)))


def test_quartic_workload_as_terms_follows_the_quartic_model():
    G, mu2 = 100.0, (0.2, 0.1, 0.0)
    q = Case("q", 3, 64, 2, 10.0, 0.01, G=(0.0, G, 0.0), mu2=mu2, expansion=True, seed=85)
    p = Case("p", 3, 64, 2, 10.0, 0.01, lam=0.0, expansion=True, seed=85, terms=_quartic_terms(G, mu2))
    phi, phid = q.inputs()
    out = []
    for case in (q, p):
        with case.sim(ce.CE_FP64) as s:
            s.load(phi, phid)
            s.step(150)
            out.append((s.read(), s.energies().as_dict(2)))
    for k in range(2):
        for i in range(2):
            assert site_error(out[1][0][k][i], out[0][0][k][i]) <= 1e-12
    for key in ("a", "rho", "pot"):
        assert abs(out[1][1][key] - out[0][1][key]) <= 1e-12 * abs(out[0][1][key])


def test_polynomial_pool_members_match_lone_runs_bitwise():
    cases = [(Case("p64", 3, 64, 2, 10.0, 0.01, lam=0.0, expansion=True, kappa=KAPPA, seed=86, terms=SEXTIC), 40),
             (Case("p256", 2, 256, 3, 40.0, 0.01, lam=0.0, seed=87, terms=TRILINEAR), 33),
             (Case("q64", 3, 64, 2, 10.0, 0.01, G=(0.0, 100.0, 0.0), expansion=True, seed=88), 27)]
    with ce.Pool(16 << 30) as pool:
        ids = []
        for case, steps in cases:
            phi, phid = case.inputs()
            ids.append(pool.admit(case.params(), phi, phid, steps))
        while pool.info().active > 0:
            pool.run_block(10)
        res = [pool.retire(j) for j in ids]
    for (case, steps), (pf, pfd) in zip(cases, res):
        cfg = ce.ce_pool_launch_for(case.params())
        phi, phid = case.inputs()
        with case.sim(ce.CE_FP32) as s:
            s.set_launch(*cfg.as_tuple())
            s.load(phi, phid)
            s.step(steps)
            f, fd = s.read()
        assert np.array_equal(f, pf) and np.array_equal(fd, pfd), case.name


def test_polynomial_grid_image_resumes_bitwise():
    case = Case("img", 3, 32, 2, 5.0, 0.01, lam=0.0, expansion=True, kappa=KAPPA, seed=89, terms=SEXTIC)
    phi, phid = case.inputs()
    with case.sim(ce.CE_FP32) as s:
        s.load(phi, phid)
        s.step(30)
        img = ce.ce_save_image(s.handle)
        s.step(25)
        want = s.read()
    p = ce.ce_image_params(img)
    assert p.model == ce.CE_MODEL_POLYNOMIAL and p.nterms == len(SEXTIC)
    with ce.Simulation.from_image(img) as r:
        r.step(25)
        got = r.read()
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_stiff_polynomial_is_refused_at_start():
    # a sixth-order term large enough that the curvature at the loaded fields
    # breaks the leapfrog limit dt sqrt(4 d/dx^2 + m^2) < 2
    case = Case("stiff", 3, 16, 1, 4.0, 0.05, lam=0.0, seed=90, background=(2.0, 0.0, 0.0),
                terms=((5.0, (6, 0, 0)),))
    phi, phid = case.inputs()
    with case.sim(ce.CE_FP32) as s:
        with pytest.raises(ce.CeError) as ei:
            s.load(phi, phid)
        assert ei.value.status == ce.CE_EINVAL and "unstable" in str(ei.value)
