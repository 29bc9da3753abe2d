"""Scheduling of the continuous-batching server, on the CPU with a fake pool.

The fake pool keeps the C pool's contract (byte budget with CE_EBUSY,
members advancing min(k, steps left) per block, poll/retire, non-finite
members reported by poll) and simulates device time, so admission order,
budget limits, continuous joining, failure isolation and the latency
arithmetic are checked without a GPU.
"""
import threading
import time

import numpy as np
import pytest

from paper_0712_0813_amd import ce
from paper_0712_0813_amd.serve import JobRecord, Server, summarize, _percentile
from paper_0712_0813_amd.workloads import Job, Lattice, serving_mix


class FakeEnergy:
    def __init__(self, step):
        self.step = step

    def as_dict(self, nf):
        return {"step": self.step}


class FakePool:
    RATE = 1e8  # simulated site-field updates/s

    def __init__(self, budget):
        self.budget = budget
        self.used = 0
        self.next = 1
        self.m = {}
        self.max_members = 0
        self.admit_order = []
        self.blocks = 0
        self.lock = threading.Lock()   # admissions come from another thread

    def __enter__(self):
        return self

    def __exit__(self, *a):
        pass

    @staticmethod
    def bytes_of(p):
        return 16 * p.nfields * p.N ** p.dims + 4096

    def admit(self, p, phi, phid, nsteps, launch=None):
        with self.lock:
            return self._admit(p, phi, phid, nsteps)

    def _admit(self, p, phi, phid, nsteps):
        b = self.bytes_of(p)
        if b > self.budget:
            raise ce.CeError(ce.CE_EINVAL, "larger than the whole budget")
        if self.used + b > self.budget:
            raise ce.CeError(ce.CE_EBUSY, "over budget")
        pid = self.next
        self.next += 1
        self.m[pid] = {"left": nsteps, "work": p.nfields * p.N ** p.dims, "bytes": b, "step": 0,
                       "bad": bool(np.isnan(phi).any())}
        self.used += b
        self.max_members = max(self.max_members, len(self.m))
        self.admit_order.append(pid)
        return pid

    def set_quota(self, pid, q):
        with self.lock:
            self.m[pid]["quota"] = q

    def run_block(self, k):
        work = 0
        with self.lock:
            for v in self.m.values():
                adv = min(k, v["left"])
                if v.get("quota", -1) >= 0:
                    adv = min(adv, v["quota"])
                v["left"] -= adv
                v["step"] += adv
                work += adv * v["work"]
            self.blocks += 1
        time.sleep(work / self.RATE)

    def steps_left(self, pid):
        return self.m[pid]["left"]

    def poll(self, pid, want_energy=True, allow_nonfinite=False):
        v = self.m[pid]
        if want_energy and v["bad"]:
            raise ce.CeError(ce.CE_ENONFINITE, "non-finite")
        return v["left"] == 0, (FakeEnergy(v["step"]) if want_energy else None)

    def retire(self, pid, read=True):
        with self.lock:
            self.used -= self.m[pid]["bytes"]
            del self.m[pid]
        return None, None

    def info(self):
        class I:
            pass
        i = I()
        with self.lock:
            i.active = sum(v["left"] > 0 for v in self.m.values())
            i.members = len(self.m)
            i.used_bytes = self.used
        return i


def _jobs(n, spacing, N=16, steps=100, dims=3, bad=()):
    out = []
    for i in range(n):
        lat = Lattice(f"j{i}", dims=dims, N=N, nfields=2, L=10.0, dt=0.01, steps=steps,
                      G=(0.0, 10.0, 0.0), seed=i)
        out.append(Job(i, i * spacing, lat))
    return out


def _inputs_fn(bad):
    def make(lat):
        shape = (lat.nfields,) + (lat.N,) * lat.dims
        phi = np.zeros(shape)
        if lat.seed in bad:
            phi[0, 0] = np.nan
        return phi, np.zeros(shape)
    return make


def test_all_jobs_complete_in_arrival_order_with_continuous_joining():
    pools = []

    def factory(budget):
        p = FakePool(budget)
        pools.append(p)
        return p

    jobs = _jobs(12, 0.01, steps=300)
    srv = Server(budget_bytes=1 << 40, block_ms=2.0, workers=2, pool_factory=factory,
                 make_inputs=_inputs_fn(()), admit_threads=1)
    recs = srv.run(jobs)
    assert all(r.status == "done" for r in recs)
    assert all(r.energy["step"] == 300 for r in recs)
    p = pools[0]
    assert p.admit_order == sorted(p.admit_order)
    assert p.max_members > 1          # jobs overlapped on the device
    for r in recs:
        assert r.arrival <= r.ready <= r.admitted <= r.finished <= r.done


def test_budget_limits_concurrency_and_queues():
    pools = []

    def factory(budget):
        p = FakePool(budget)
        pools.append(p)
        return p

    jobs = _jobs(10, 0.0, N=16, steps=200)
    one = FakePool.bytes_of(ce.make_params(3, 16, 2, 10.0, 0.01))
    srv = Server(budget_bytes=3 * one, block_ms=1.0, workers=4, pool_factory=factory,
                 make_inputs=_inputs_fn(()))
    recs = srv.run(jobs)
    assert all(r.status == "done" for r in recs)
    assert pools[0].max_members <= 3
    # later jobs waited in the queue for memory, and the server saw it
    assert max(r.admitted - r.ready for r in recs) > 0
    assert srv.waited_for_memory > 0
    assert one <= srv.peak_used_bytes <= 3 * one


def test_failed_job_is_isolated():
    jobs = _jobs(6, 0.005, steps=120)
    srv = Server(budget_bytes=1 << 40, block_ms=1.0, workers=2,
                 pool_factory=lambda b: FakePool(b), make_inputs=_inputs_fn({3}))
    recs = srv.run(jobs)
    assert recs[3].status == "failed"
    assert all(r.status == "done" for i, r in enumerate(recs) if i != 3)


def test_job_larger_than_the_whole_budget_fails_and_the_run_ends():
    """A member that can never fit the budget is refused with CE_EINVAL (not
    CE_EBUSY, which would make the admitter wait for a retirement forever):
    that job fails, the others finish and run() returns."""
    jobs = _jobs(5, 0.005, N=16, steps=80)
    big = Lattice("big", dims=3, N=32, nfields=2, L=10.0, dt=0.01, steps=80, G=(0.0, 10.0, 0.0), seed=99)
    jobs.insert(2, Job(99, 0.006, big))
    one = FakePool.bytes_of(ce.make_params(3, 16, 2, 10.0, 0.01))
    assert FakePool.bytes_of(ce.make_params(3, 32, 2, 10.0, 0.01)) > 3 * one
    srv = Server(budget_bytes=3 * one, block_ms=1.0, workers=2, pool_factory=lambda b: FakePool(b),
                 make_inputs=_inputs_fn(()), admit_threads=2)
    done = []
    th = threading.Thread(target=lambda: done.append(srv.run(jobs)), daemon=True)
    th.start()
    th.join(60)
    assert not th.is_alive(), "the server hung on a job larger than its budget"
    recs = {r.job_id: r for r in done[0]}
    assert recs[99].status == "failed"
    assert all(r.status == "done" for jid, r in recs.items() if jid != 99)


def test_summary_percentiles():
    recs = []
    for i in range(100):
        r = JobRecord(i, 1e9, 0.0, 0.1, 0.2, 1.0 + i, 1.0 + i)
        r.status = "done"
        recs.append(r)
    s = summarize(recs, makespan=200.0)
    assert s["p50_latency_s"] == pytest.approx(np.percentile(np.arange(1.0, 101.0), 50))
    assert s["p99_latency_s"] == pytest.approx(np.percentile(np.arange(1.0, 101.0), 99))
    assert s["site_field_updates_per_s"] == pytest.approx(100 * 1e9 / 200.0)
    assert s["breakdown_mean_s"]["host_init"] == pytest.approx(0.1)
    assert np.isnan(_percentile([], 50))


def test_serving_mix_shape():
    jobs = serving_mix(2000)
    assert len(jobs) == 2000
    arr = np.array([j.arrival for j in jobs])
    assert np.all(np.diff(arr) >= 0)
    assert 80 < arr[-1] < 120           # Poisson at 20/s
    d3 = [j for j in jobs if j.lattice.dims == 3]
    assert 0.7 < len(d3) / 2000 < 0.8
    assert {j.lattice.N for j in d3} == {32, 64, 128, 256}
    assert {j.lattice.N for j in jobs if j.lattice.dims == 2} == {256, 512, 1024, 2048}
    assert {j.lattice.nfields for j in jobs} == {1, 2, 3}
    assert all(200 <= j.lattice.steps <= 2000 for j in jobs)
    G = np.array([g for j in jobs for g in j.lattice.G[1:j.lattice.nfields]])
    assert G.min() >= 1.0 and G.max() <= 1e4
    # every job is leapfrog-stable at its couplings
    for j in jobs:
        lat = j.lattice
        m2 = max([3.0] + [lat.G[k] for k in range(1, lat.nfields)])
        assert lat.dt * np.sqrt(4 * lat.dims / lat.dx ** 2 + m2) < 2


def test_short_first_lets_small_jobs_through():
    # one long job and a few short ones arriving just after it: with
    # shortest-first budgets the short ones finish much sooner than under
    # plain processor sharing, and everything still completes
    class Fast(FakePool):
        RATE = 1e9

    big = Lattice("big", dims=3, N=32, nfields=2, L=10.0, dt=0.01, steps=2000, G=(0.0, 10.0, 0.0), seed=0)
    jobs = [Job(0, 0.0, big)]
    for i in range(4):
        small = Lattice(f"s{i}", dims=3, N=8, nfields=1, L=2.5, dt=0.01, steps=1000, seed=i + 1)
        jobs.append(Job(i + 1, 0.03 + 0.002 * i, small))
    worst_small = {}
    for short_first in (True, False):
        srv = Server(budget_bytes=1 << 40, block_ms=5.0, workers=2, pool_factory=lambda b: Fast(b),
                     make_inputs=_inputs_fn(()), short_first=short_first, rate_guess=Fast.RATE)
        recs = srv.run(jobs)
        assert all(r.status == "done" for r in recs)
        assert all(r.energy["step"] == j.lattice.steps for r, j in zip(recs, jobs))
        worst_small[short_first] = max(r.latency for r in recs[1:])
    assert worst_small[True] < 0.5 * worst_small[False], worst_small


class RecordingPool(FakePool):
    """FakePool that remembers retirements: (pool id, steps left, read)."""

    def __init__(self, budget):
        super().__init__(budget)
        self.retired = []

    def retire(self, pid, read=True):
        self.retired.append((pid, self.m[pid]["left"], read))
        return super().retire(pid, read)


def _serve_with_cancels(jobs, cancels, budget=1 << 40, **kw):
    """Run jobs; cancels = [(seconds after start, job id)] issued from a timer thread."""
    pools = []

    def factory(b):
        p = RecordingPool(b)
        pools.append(p)
        return p

    srv = Server(budget_bytes=budget, block_ms=1.0, workers=2, pool_factory=factory,
                 make_inputs=_inputs_fn(()), **kw)
    timers = [threading.Timer(t, srv.cancel, args=(jid,)) for t, jid in cancels]
    for tm in timers:
        tm.start()
    recs = srv.run(jobs)
    for tm in timers:
        tm.join()
    return recs, pools[0]


def test_cancel_running_job_frees_its_memory_and_others_finish():
    # job 0 is long (about 2 s of simulated device time alone) and is
    # cancelled while it runs; the short jobs around it complete
    jobs = _jobs(5, 0.01, steps=100)
    long = Lattice("long", dims=3, N=16, nfields=2, L=10.0, dt=0.01, steps=30000, G=(0.0, 10.0, 0.0), seed=99)
    jobs[0] = Job(0, 0.0, long)
    recs, pool = _serve_with_cancels(jobs, [(0.3, 0)])
    assert recs[0].status == "cancelled"
    assert all(r.status == "done" for r in recs[1:])
    assert all(r.energy["step"] == 100 for r in recs[1:])
    left = {pid: (n, read) for pid, n, read in pool.retired}
    first = pool.admit_order[0]
    assert left[first][0] > 0 and left[first][1] is False   # retired mid-run, nothing read back
    assert pool.used == 0 and not pool.m
    s = summarize(recs, makespan=1.0)
    assert s["cancelled"] == 1 and s["completed"] == 4


def test_cancel_before_arrival_is_never_admitted():
    jobs = _jobs(4, 0.2, steps=50)
    recs, pool = _serve_with_cancels(jobs, [(0.05, 3)])
    assert recs[3].status == "cancelled"
    assert [r.status for r in recs[:3]] == ["done"] * 3
    assert len(pool.admit_order) == 3


def test_cancel_job_waiting_for_memory():
    # the budget holds one member; job 1 waits behind the long job 0 and is
    # cancelled while it waits: it is never admitted, and job 2 runs after 0
    one = FakePool.bytes_of(ce.make_params(3, 16, 2, 10.0, 0.01))
    jobs = _jobs(3, 0.01, steps=6000)   # about 0.5 s each
    recs, pool = _serve_with_cancels(jobs, [(0.05, 1)], budget=one)
    assert [r.status for r in recs] == ["done", "cancelled", "done"]
    assert len(pool.admit_order) == 2 and pool.max_members == 1


def test_cancel_after_completion_keeps_result():
    jobs = _jobs(2, 0.0, steps=20)
    srv = Server(budget_bytes=1 << 40, block_ms=1.0, workers=2, pool_factory=lambda b: FakePool(b),
                 make_inputs=_inputs_fn(()))
    recs = srv.run(jobs)
    assert srv.cancel(0) is False      # no run in progress: nothing recorded
    assert all(r.status == "done" for r in recs)
    # the server is reusable, and a stale request does not reach the next run
    assert all(r.status == "done" for r in srv.run(jobs))


def test_cancel_of_unknown_job_is_ignored():
    jobs = _jobs(3, 0.01, steps=50)
    recs, pool = _serve_with_cancels(jobs, [(0.02, 77)])
    assert all(r.status == "done" for r in recs)
