"""Device-generated initial conditions (ce_generate_fields) against the
oracle's generator (same Philox stream, same definition), then evolved
against the oracle run from the oracle's arrays."""
import time

import numpy as np
import pytest

from paper_0712_0813_amd import ce
from oracle import Oracle, grf_field, grf_initial, grf_mode_parts, grf_sites
from _parity import TOL_MEAN, TOL_SITE, Case, energy_errors, site_error

pytestmark = pytest.mark.gpu

CASES = [
    (Case("3d_64_exp", 3, 64, 2, 10.0, 0.01, G=(0.0, 100.0, 0.0), expansion=True, seed=41), ce.CE_FP64),
    (Case("3d_32_3f", 3, 32, 3, 10.0, 0.01, G=(0.0, 100.0, 30.0), seed=42), ce.CE_FP32),
    (Case("3d_8_chunked", 3, 8, 1, 4.0, 0.01, seed=43), ce.CE_FP32),
    (Case("3d_4_tiny", 3, 4, 1, 2.0, 0.01, seed=44), ce.CE_FP32),
    (Case("2d_256", 2, 256, 2, 40.0, 0.01, G=(0.0, 100.0, 0.0), seed=45), ce.CE_FP64),
    (Case("2d_2048", 2, 2048, 1, 200.0, 0.02, seed=46), ce.CE_FP32),
    (Case("1d_1024", 1, 1024, 2, 100.0, 0.02, G=(0.0, 10.0, 0.0), seed=47), ce.CE_FP64),
]


def spec_of(case, bg=(1.0, 0.0, 0.0), bgdot=(0.0, 0.0, 0.0)):
    return ce.make_init_spec(case.seed, case.m_eff2(), case.amp, bg, bgdot)


@pytest.mark.parametrize("case,precision", CASES, ids=[c[0].name for c in CASES])
def test_generated_fields_match_oracle_generator(case, precision):
    bg, bgdot = (1.0, 0.0, 0.0), (0.0, 0.02, -0.01)
    print(f"[gen] {case.name}", flush=True)
    phi, phid = grf_initial(case.seed, case.dims, case.N, case.L, case.nfields, case.m_eff2(), case.amp,
                            bg, bgdot)
    steps = 0 if case.N >= 2048 else 200
    with case.sim(precision) as s:
        s.generate(spec_of(case, bg, bgdot))
        f0, fd0 = s.read()
        s.step(steps)
        f, fd = s.read()
        log = [e.as_dict(case.nfields) for e in s.energy_log(steps + 1)]
    # the generated field itself (f at step 0 is phi at tau = 0): FP64 to
    # rounding of the transforms; FP32 storage adds one rounding of the
    # deviation (at most 2^-24 of it)
    for i in range(case.nfields):
        d_gpu = f0[i] - bg[i]
        d_orc = phi[i] - bg[i]
        rms = np.sqrt(np.mean(d_orc ** 2))
        assert rms > 0
        bound = 1e-12 * rms + (0.0 if precision == ce.CE_FP64 else 2.0 ** -24 * np.abs(d_orc))
        assert np.all(np.abs(d_gpu - d_orc) <= bound), i
    orc = Oracle(case.oracle_params(), phi, phid)
    for i in range(case.nfields):   # derivative at dt/2 after the start-up half step
        assert site_error(fd0[i], orc.pi[i]) <= TOL_SITE[precision]
    if steps == 0:
        return
    orc.step(steps)
    for i in range(case.nfields):
        assert site_error(f[i], orc.f[i]) <= TOL_SITE[precision]
        assert site_error(fd[i], orc.pi[i]) <= TOL_SITE[precision]
    for g, o in zip(log, orc.log):
        errs = energy_errors(g, o, case.nfields)
        worst = max(errs, key=errs.get)
        assert errs[worst] <= TOL_MEAN[precision], (g["step"], worst, errs[worst])


def test_generation_is_deterministic_and_seeded():
    case = Case("det", 3, 32, 2, 10.0, 0.01, G=(0.0, 100.0, 0.0), seed=50)
    out = []
    for seed in (50, 50, 51):
        with case.sim(ce.CE_FP32) as s:
            s.generate(ce.make_init_spec(seed, case.m_eff2(), case.amp))
            out.append(s.read())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert not np.array_equal(out[0][0], out[2][0])


def test_generation_rejections():
    case = Case("rej", 3, 32, 1, 10.0, 0.01, seed=52)
    with case.sim(ce.CE_FP32) as s:
        bad = spec_of(case)
        bad.amp = -1.0
        with pytest.raises(ce.CeError) as e:
            s.generate(bad)
        assert e.value.status == ce.CE_EINVAL
        bad = spec_of(case)
        bad.m_eff2[0] = float("nan")
        with pytest.raises(ce.CeError):
            s.generate(bad)
        s.generate(spec_of(case))
        with pytest.raises(ce.CeError) as e:
            s.generate(spec_of(case))
        assert e.value.status == ce.CE_ESTATE
    odd = Case("odd", 3, 24, 1, 10.0, 0.01, seed=53)
    with odd.sim(ce.CE_FP32) as s:
        with pytest.raises(ce.CeError) as e:
            s.generate(spec_of(odd))
        assert e.value.status == ce.CE_EINVAL and "power of two" in str(e.value)
    # an unstable generated state is rejected, and the simulation takes a
    # stable one afterwards
    stiff = Case("stiff", 3, 16, 2, 10.0, 0.01, G=(0.0, 1e6, 0.0), seed=54)
    with stiff.sim(ce.CE_FP32) as s:
        with pytest.raises(ce.CeError) as e:
            s.generate(spec_of(stiff))
        assert "unstable" in str(e.value)
        s.generate(ce.make_init_spec(54, stiff.m_eff2(), 1e-3, (0.0, 0.0, 0.0)))
        s.step(3)


def test_pool_member_generated_equals_lone_generated():
    case = Case("pool", 3, 64, 2, 10.0, 0.01, G=(0.0, 100.0, 0.0), expansion=True, seed=55)
    params = ce.make_params(3, 64, 2, 10.0, 0.01, G=case.G, expansion=True, kappa=case.kappa)
    launch = ce.ce_pool_launch_for(params).as_tuple()
    with ce.Pool(1 << 30) as pool:
        j = pool.admit_generated(params, spec_of(case), 60)
        while not pool.poll(j, want_energy=False)[0]:
            pool.run_block(20)
        done, e = pool.poll(j)
        f_pool, fd_pool = pool.retire(j)
    with case.sim(ce.CE_FP32) as s:
        s.set_launch(*launch)
        s.generate(spec_of(case))
        s.step(60)
        f, fd = s.read()
        e_lone = s.energies()
    assert np.array_equal(f, f_pool) and np.array_equal(fd, fd_pool)
    assert e.as_dict(2) == e_lone.as_dict(2)


def _parseval(re, im):
    """sum |H_n|^2 over the mode box, H_n = (c_n + conj(c_-n)) / 2: the
    volume mean of delta^2 for delta = Re sum_n c_n exp(2 pi i n.x/N)."""
    hr = 0.5 * (re + re[(slice(None, None, -1),) * re.ndim])
    hi = 0.5 * (im - im[(slice(None, None, -1),) * im.ndim])
    return float(np.sum(hr * hr) + np.sum(hi * hi))


def test_full_size_generation_sampled_sites():
    """The 1024^3 two-field workload as the benchmark generates it (seed 1).
    All four arrays against the oracle's modes: the step-0 diagnostics give
    <phi_i> (the background: the band has no n = 0 mode), <phi_i^2> and
    K_i(0) = 1/2 <phidot_i^2> (formed before the start-up half kick), which
    Parseval fixes as sums over the oracle's modes; 16 sites of each field
    array against the oracle's direct sum over every mode of the band.  (The
    stored derivative already holds the half kick, so derivative arrays are
    checked through K_i(0).)"""
    from concurrent.futures import ThreadPoolExecutor
    from paper_0712_0813_amd.workloads import LATTICE1024_EXPANDING as W
    t0 = time.time()
    rng = np.random.default_rng(7)
    nsite = 16
    sites = rng.integers(0, W.N ** 3, nsite)
    with ce.Simulation.from_lattice(W, precision=ce.CE_FP32) as s:
        s.generate(ce.lattice_init_spec(W))
        e0 = s.energies().as_dict(W.nfields)
        got = [s.read_sites(i, sites)[0] for i in range(W.nfields)]
        print(f"[gen] 1024^3 generated ({time.time() - t0:.1f} s)", flush=True)
    meff = W.m_eff2()

    def oracle_array(i, kind):
        re, im = grf_mode_parts(W.seed, i, kind, 3, W.N, W.L, W.amp, meff[i])
        return re, im, _parseval(re, im)

    with ThreadPoolExecutor(4) as ex:
        arrays = {(i, k): ex.submit(oracle_array, i, k) for i in range(W.nfields) for k in (0, 1)}
        parseval = {key: f.result()[2] for key, f in arrays.items()}
        print(f"[gen] oracle modes and Parseval sums done ({time.time() - t0:.1f} s)", flush=True)
        # direct sums at the sampled sites, one task per (field, site)
        sums = {(i, j): ex.submit(grf_sites, arrays[(i, 0)].result()[0], arrays[(i, 0)].result()[1], W.N,
                                  sites[j:j + 1])
                for i in range(W.nfields) for j in range(nsite)}
        ref = [np.concatenate([sums[(i, j)].result() for j in range(nsite)]) for i in range(W.nfields)]
        print(f"[gen] oracle sites done ({time.time() - t0:.1f} s)", flush=True)
    del arrays
    for i in range(W.nfields):
        b = W.background[i]
        # the stored deviation is FP32: each site within one rounding of it
        d = got[i] - b
        assert np.max(np.abs(d - ref[i])) <= 1e-6 * np.max(np.abs(ref[i])) + 1e-12, (i, d, ref[i])
        var_f, var_d = parseval[(i, 0)], parseval[(i, 1)]
        rms = np.sqrt(var_f)
        assert abs(e0["mean"][i] - b) <= 1e-6 * rms, (i, e0["mean"][i], b)
        # <phi^2> = b^2 + 2 b <delta> + <delta^2>, and <delta> = 0
        assert abs((e0["mean_sq"][i] - b * b) - var_f) <= 1e-5 * var_f + 2e-6 * abs(b) * rms, \
            (i, e0["mean_sq"][i] - b * b, var_f)
        assert abs(2.0 * e0["kin"][i] - var_d) <= 1e-5 * var_d, (i, 2.0 * e0["kin"][i], var_d)
        print(f"[gen] field {i}: <delta^2> {e0['mean_sq'][i] - b * b:.9e} vs {var_f:.9e}, "
              f"<deltadot^2> {2 * e0['kin'][i]:.9e} vs {var_d:.9e}", flush=True)
