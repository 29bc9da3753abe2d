"""The pool (batched ensembles / serving) against lone simulations and the oracle.

A member must give bitwise the same fields and diagnostics as the same lattice
run alone with ce_pool_launch_for's launch configuration, whatever else is in
the pool, including members of other classes and members finishing mid-block.
"""
import numpy as np
import pytest

from paper_0712_0813_amd import ce
from _parity import TOL_MEAN, TOL_SITE, Case, energy_errors, site_error
from oracle import Oracle

pytestmark = pytest.mark.gpu

MIX = [
    (Case("p_cube32", 3, 32, 2, 10.0, 0.01, G=(0.0, 100.0, 0.0), seed=21), 37),
    (Case("p_cube64_exp", 3, 64, 2, 10.0, 0.01, G=(0.0, 300.0, 0.0), expansion=True, seed=22), 50),
    (Case("p_cube64_1f", 3, 64, 1, 10.0, 0.01, mu2=(0.3, 0.0, 0.0), expansion=True, seed=23), 64),
    (Case("p_cube48_direct", 3, 48, 2, 7.5, 0.01, G=(0.0, 50.0, 0.0), seed=24), 29),
    (Case("p_square128_3f", 2, 128, 3, 20.0, 0.01, G=(0.0, 40.0, 900.0), expansion=True, seed=25), 45),
    (Case("p_line256", 1, 256, 2, 40.0, 0.01, G=(0.0, 20.0, 0.0), seed=26), 64),
    (Case("p_cube64_exp_b", 3, 64, 2, 10.0, 0.01, G=(0.0, 3000.0, 0.0), expansion=True, seed=27), 16),
    (Case("p_square256_stream", 2, 256, 2, 40.0, 0.01, G=(0.0, 500.0, 0.0), expansion=True, seed=28), 33),
    (Case("p_square512_1f", 2, 512, 1, 80.0, 0.01, mu2=(0.1, 0.0, 0.0), seed=29), 20),
]


def _params(case, precision=ce.CE_FP32):
    return ce.make_params(case.dims, case.N, case.nfields, case.L, case.dt, lam=case.lam, G=case.G,
                          mu2=case.mu2, expansion=case.expansion, kappa=case.kappa,
                          precision=precision)


def _alone(case, steps, precision=ce.CE_FP32):
    phi, phid = case.inputs()
    cfg = ce.ce_pool_launch_for(_params(case, precision))
    with case.sim(precision) as s:
        s.set_launch(*cfg.as_tuple())
        s.load(phi, phid)
        s.step(steps)
        f, fd = s.read()
        log = [e.as_dict(case.nfields) for e in s.energy_log(steps + 1)]
    return f, fd, log


@pytest.mark.parametrize("precision", [ce.CE_FP32, ce.CE_FP64], ids=["fp32", "fp64"])
def test_pool_members_match_lone_runs_bitwise(precision):
    res = {}
    with ce.Pool(64 << 30) as pool:
        ids = {}
        for case, steps in MIX:
            phi, phid = case.inputs()
            ids[case.name] = pool.admit(_params(case, precision), phi, phid, steps)
        assert pool.info().members == len(MIX)
        blocks = 0
        while pool.info().active > 0:
            pool.run_block(7)  # members finish mid-block
            blocks += 1
            assert blocks < 100
        for case, steps in MIX:
            done, e = pool.poll(ids[case.name])
            assert done and e.step == steps
            f, fd = pool.retire(ids[case.name])
            res[case.name] = (f, fd, e.as_dict(case.nfields))
        assert pool.info().members == 0 and pool.info().used_bytes == 0
    for case, steps in MIX:
        f, fd, log = _alone(case, steps, precision)
        pf, pfd, pe = res[case.name]
        assert np.array_equal(pf, f), case.name
        assert np.array_equal(pfd, fd), case.name
        assert pe == log[-1], case.name


ORACLE_MIX = MIX[:5] + MIX[7:8]


def test_pool_members_match_oracle():
    with ce.Pool(16 << 30) as pool:
        ids = {}
        for case, steps in ORACLE_MIX:
            phi, phid = case.inputs()
            ids[case.name] = pool.admit(_params(case), phi, phid, steps)
        while pool.info().active > 0:
            pool.run_block(16)
        for case, steps in ORACLE_MIX:
            phi, phid = case.inputs()
            orc = Oracle(case.oracle_params(), phi, phid)
            orc.step(steps)
            done, e = pool.poll(ids[case.name])
            f, fd = pool.retire(ids[case.name])
            for i in range(case.nfields):
                assert site_error(f[i], orc.f[i]) <= TOL_SITE[ce.CE_FP32]
                assert site_error(fd[i], orc.pi[i]) <= TOL_SITE[ce.CE_FP32]
            errs = energy_errors(e.as_dict(case.nfields), orc.state, case.nfields)
            assert max(errs.values()) <= TOL_MEAN[ce.CE_FP32], (case.name, errs)


def test_pool_budget_and_admission_between_blocks():
    case, _ = MIX[1]
    p = _params(case)
    one = ce.ce_required_bytes(p)
    phi, phid = case.inputs()
    with ce.Pool(int(2.5 * one)) as pool:
        a = pool.admit(p, phi, phid, 20)
        b = pool.admit(p, phi, phid, 40)
        with pytest.raises(ce.CeError) as ei:
            pool.admit(p, phi, phid, 10)
        assert ei.value.status == ce.CE_EBUSY
        pool.run_block(20)
        assert pool.poll(a)[0] and not pool.poll(b)[0]
        pool.retire(a, read=False)
        c = pool.admit(p, phi, phid, 20)   # joins while b is half way
        pool.run_block(20)
        assert pool.poll(b)[0] and pool.poll(c)[0]
        fb, _ = pool.retire(b)
        fc, _ = pool.retire(c)
    # b ran 40 steps and c 20 steps of the same lattice
    f40, _, _ = _alone(case, 40)
    f20, _, _ = _alone(case, 20)
    assert np.array_equal(fb, f40) and np.array_equal(fc, f20)


def test_admissions_from_another_thread_bitwise():
    # one thread admits while this one keeps enqueuing blocks; every member
    # still matches its lone run bitwise, whenever it joined
    import threading
    import time
    inputs = {case.name: case.inputs() for case, _ in MIX}
    ids = {}
    errors = []
    with ce.Pool(64 << 30) as pool:
        def admitter():
            try:
                for case, steps in MIX:
                    phi, phid = inputs[case.name]
                    ids[case.name] = pool.admit(_params(case), phi, phid, steps)
                    time.sleep(0.003)
            except Exception as e:  # reported below
                errors.append(e)
        th = threading.Thread(target=admitter)
        th.start()
        try:
            blocks = 0
            t_end = time.perf_counter() + 120.0
            while th.is_alive() or pool.info().active > 0:
                if pool.info().active == 0:
                    time.sleep(0.001)   # waiting for the next admission
                    continue
                pool.run_block(5)
                blocks += 1
                assert time.perf_counter() < t_end
        finally:
            th.join()   # the pool must outlive every admission
        assert not errors, errors
        res = {}
        for case, steps in MIX:
            done, e = pool.poll(ids[case.name])
            assert done and e.step == steps
            res[case.name] = pool.retire(ids[case.name]) + (e.as_dict(case.nfields),)
    for case, steps in MIX:
        f, fd, log = _alone(case, steps)
        pf, pfd, pe = res[case.name]
        assert np.array_equal(pf, f) and np.array_equal(pfd, fd), case.name
        assert pe == log[-1], case.name


def test_enqueued_blocks_steps_left_and_memory_reuse():
    case, _ = MIX[1]
    p = _params(case)
    phi, phid = case.inputs()
    with ce.Pool(8 << 30) as pool:
        a = pool.admit(p, phi, phid, 25)
        # three blocks enqueued back to back (the pool lets two be in flight)
        pool.run_block(10)
        assert pool.steps_left(a) == 15
        pool.run_block(10)
        pool.run_block(10)
        assert pool.steps_left(a) == 0
        done, e = pool.poll(a)
        assert done and e.step == 25
        f1, fd1 = pool.retire(a)
        used = pool.info().used_bytes
        # the next member of the same size reuses the retired memory
        b = pool.admit(p, phi, phid, 25)
        assert pool.info().used_bytes == used + ce.ce_required_bytes(p)
        while pool.info().active > 0:
            pool.run_block(7)
        f2, fd2 = pool.retire(b)
    fa, fda, _ = _alone(case, 25)
    assert np.array_equal(f1, fa) and np.array_equal(fd1, fda)
    assert np.array_equal(f2, fa) and np.array_equal(fd2, fda)


def test_admit_with_launch_matches_lone_run():
    case, steps = MIX[1]
    cfg = (ce.CE_KERNEL_TILED3D, 4, 16, 256, 32, 8)
    phi, phid = case.inputs()
    with ce.Pool(8 << 30) as pool:
        j = pool.admit(_params(case), phi, phid, steps, launch=cfg)
        while pool.info().active > 0:
            pool.run_block(16)
        pf, pfd = pool.retire(j)
    with case.sim(ce.CE_FP32) as s:
        s.set_launch(*cfg)
        s.load(phi, phid)
        s.step(steps)
        f, fd = s.read()
    assert np.array_equal(pf, f) and np.array_equal(pfd, fd)


def test_quotas_pause_and_limit_members_bitwise():
    # per-block step budgets change when a member's steps run, never what
    # they compute
    a_case, _ = MIX[1]
    b_case, _ = MIX[7]       # 2-D streaming class
    pa, pb = _params(a_case), _params(b_case)
    ia, ib = a_case.inputs(), b_case.inputs()
    with ce.Pool(16 << 30) as pool:
        a = pool.admit(pa, *ia, 30)
        b = pool.admit(pb, *ib, 30)
        pool.set_quota(a, 3)
        pool.set_quota(b, 0)          # paused
        pool.run_block(10)
        assert pool.steps_left(a) == 27 and pool.steps_left(b) == 30
        pool.set_quota(b, -1)
        pool.run_block(10)
        assert pool.steps_left(a) == 24 and pool.steps_left(b) == 20
        pool.set_quota(a, -1)
        while pool.info().active > 0:
            pool.run_block(10)
        ea = pool.poll(a)[1].as_dict(a_case.nfields)
        eb = pool.poll(b)[1].as_dict(b_case.nfields)
        fa, fda = pool.retire(a)
        fb, fdb = pool.retire(b)
    for case, f, fd, e in ((a_case, fa, fda, ea), (b_case, fb, fdb, eb)):
        lf, lfd, log = _alone(case, 30)
        assert np.array_equal(f, lf) and np.array_equal(fd, lfd), case.name
        assert e == log[-1], case.name


def test_nonfinite_member_is_reported_and_isolated():
    # one member overflows FP32 at once; it reports CE_ENONFINITE with the
    # step it went bad at, and its neighbours in the same launches still end
    # bitwise where their lone runs end
    bad_case, steps = MIX[1]
    phi, phid = bad_case.inputs()
    phid = phid.copy()
    phid[1, 3, 4, 5] = 1e30
    with ce.Pool(8 << 30) as pool:
        jb = pool.admit(_params(bad_case), phi, phid, steps)
        good = {}
        for case, st in (MIX[0], MIX[2], MIX[6]):
            p, pd = case.inputs()
            good[case.name] = (case, st, pool.admit(_params(case), p, pd, st))
        while pool.info().active > 0:
            pool.run_block(9)
        with pytest.raises(ce.CeError) as ei:
            pool.poll(jb)
        assert ei.value.status == ce.CE_ENONFINITE
        done, e = pool.poll(jb, allow_nonfinite=True)
        assert done and e.step == steps
        pool.retire(jb, read=False)
        res = {}
        for name, (case, st, j) in good.items():
            done, e = pool.poll(j)
            f, fd = pool.retire(j)
            res[name] = (f, fd, e.as_dict(case.nfields))
    for name, (case, st, _) in good.items():
        f, fd, log = _alone(case, st)
        pf, pfd, pe = res[name]
        assert np.array_equal(pf, f) and np.array_equal(pfd, fd) and pe == log[-1], name
