"""Pool lifetime and admission limits on the GPU.

ce_pool_destroy must wait for admissions in progress on other threads before
it frees the pool's streams and memory, and a member that can never fit the
budget must be refused with CE_EINVAL (CE_EBUSY would tell a caller to wait
for a retirement that cannot help).
"""
import threading
import time

import pytest

from paper_0712_0813_amd import ce

pytestmark = pytest.mark.gpu


def _params(N, nfields=2, dims=3):
    return ce.make_params(dims, N, nfields, 10.0 * N / 64, 0.01, G=(0.0, 100.0, 300.0), expansion=True,
                          kappa=2.94)


def test_member_larger_than_the_whole_budget_is_refused():
    small, big = _params(64), _params(128)
    one = ce.ce_required_bytes(small)
    assert ce.ce_required_bytes(big) > 3 * one
    with ce.Pool(3 * one) as pool:
        with pytest.raises(ce.CeError) as ei:
            pool.admit_generated(big, ce.make_init_spec(5, [3.0, 100.0]), 10)
        assert ei.value.status == ce.CE_EINVAL
        info = pool.info()
        assert info.used_bytes == 0 and info.members == 0 and info.admitting == 0
        # the pool is unharmed: a member that fits runs to completion
        jid = pool.admit_generated(small, ce.make_init_spec(5, [3.0, 100.0]), 10)
        pool.run_block(10)
        done, e = pool.poll(jid)
        assert done and e.step == 10
        pool.retire(jid, read=False)


def test_destroy_waits_for_an_admission_in_progress():
    """One thread admits a large member (allocation, device generation and
    start-up take milliseconds); once ce_pool_info shows the admission inside
    the pool, this thread destroys the pool.  Destroy must return only after
    the admission has returned, and the admission must have succeeded."""
    p = _params(256, nfields=3)
    spec = ce.make_init_spec(7, [3.0, 100.0, 300.0])
    pool = ce.ce_pool_create(4 * ce.ce_required_bytes(p))
    res = {}

    def admit():
        try:
            res["id"] = ce.ce_pool_admit_generated(pool, p, spec, 5)
            res["status"] = ce.CE_OK
        except ce.CeError as e:
            res["status"] = e.status
        res["t_end"] = time.perf_counter()

    th = threading.Thread(target=admit)
    print("[pool lifetime] admission thread started", flush=True)
    th.start()
    seen = False
    deadline = time.perf_counter() + 60.0
    while th.is_alive() and time.perf_counter() < deadline:
        if ce.ce_pool_get_info(pool).admitting > 0:
            seen = True
            break
        time.sleep(1e-4)
    t0 = time.perf_counter()
    ce.ce_pool_destroy(pool)
    t1 = time.perf_counter()
    th.join(120)
    print(f"[pool lifetime] destroy took {t1 - t0:.4f} s, admission seen in progress: {seen}", flush=True)
    assert not th.is_alive()
    assert res["status"] == ce.CE_OK
    assert res["t_end"] <= t1
