"""Batched ensembles and a continuous-batching server over the C-ABI pool.

The server keeps every admitted lattice on the device between step blocks:
jobs arriving while others run are admitted at the next block boundary as
soon as the pool's byte budget allows, members that finish are read back and
retired, and their memory goes to the next jobs.  Initial conditions are
generated on the device at admission (seeded, see ce_generate_fields), or by
a host thread pool as jobs arrive.  The per-job
timeline (arrival, inputs ready, admitted, finished, read back) gives the
latency breakdown.  Every step runs in libce's kernels; this module only
schedules.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import ce
from .inputs import lattice_initial
from .workloads import Job, Lattice


def params_of(lat: Lattice, precision: int = ce.CE_FP32) -> ce.ce_params:
    return ce.make_params(lat.dims, lat.N, lat.nfields, lat.L, lat.dt, lam=lat.lam, G=lat.G,
                          mu2=lat.mu2, expansion=lat.expansion, kappa=lat.kappa,
                          precision=precision, vacuum=lat.vacuum)


def _host_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def pinned_inputs(lat: Lattice):
    """Initial conditions for one lattice, copied into page-locked host
    memory when a GPU is present, so the upload on admission runs at DMA
    rate beside the block in flight.  Returns (phi, phidot, keepalive)."""
    phi, phid = lattice_initial(lat, 1)
    try:
        import torch
        if not torch.cuda.is_available():
            return phi, phid, None
        keep = []
        out = []
        for a in (phi, phid):
            t = torch.empty(a.shape, dtype=torch.float64, pin_memory=True)
            v = t.numpy()
            v[...] = a
            keep.append(t)
            out.append(v)
        return out[0], out[1], keep
    except ImportError:
        return phi, phid, None


def generate_all(lattices: Sequence[Lattice], workers: Optional[int] = None):
    """Initial conditions for many lattices, generated in parallel on the host."""
    workers = workers or _host_workers()
    with cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda lat: lattice_initial(lat, workers=1), lattices))


@dataclass
class EnsembleResult:
    seconds: float                 # device time of the stepping (inputs resident)
    site_field_updates: float
    energies: List[dict]           # final diagnostics per lattice

    @property
    def rate(self) -> float:
        return self.site_field_updates / self.seconds


def tuned_member_launch(lat: Lattice, precision: int = ce.CE_FP32):
    """The autotuned pool-member launch for this lattice's class, if cached."""
    from . import autotune
    return autotune.lookup(lat.dims, lat.N, lat.nfields, precision, pool=True)


def run_batched(lattices: Sequence[Lattice], inputs, steps: int, block: int = 50,
                budget_bytes: int = 200 << 30, precision: int = ce.CE_FP32,
                use_tuned: bool = True) -> EnsembleResult:
    """Every lattice in one pool (autotuned member launches when cached);
    `steps` steps in blocks of `block`."""
    with ce.Pool(budget_bytes) as pool:
        ids = []
        for lat, (phi, phid) in zip(lattices, inputs):
            cfg = tuned_member_launch(lat, precision) if use_tuned else None
            ids.append(pool.admit(params_of(lat, precision), phi, phid, steps, launch=cfg))
        # admissions return with their loads and start-up passes done
        t0 = time.perf_counter()
        left = steps
        while left > 0:
            k = min(block, left)
            pool.run_block(k)
            left -= k
        for j in ids:   # each waits for the block holding the member's last step
            pool.poll(j, want_energy=False)
        el = time.perf_counter() - t0
        energies = [pool.poll(j)[1].as_dict(lat.nfields) for j, lat in zip(ids, lattices)]
        for j in ids:
            pool.retire(j, read=False)
    work = float(sum(lat.site_fields for lat in lattices)) * steps
    return EnsembleResult(el, work, energies)


def run_sequential(lattices: Sequence[Lattice], inputs, steps: int,
                   precision: int = ce.CE_FP32) -> EnsembleResult:
    """One plain simulation after another (library defaults), stepping timed."""
    el = 0.0
    energies = []
    for lat, (phi, phid) in zip(lattices, inputs):
        with ce.Simulation.from_lattice(lat, precision) as s:
            s.load(phi, phid)
            s.sync()
            t0 = time.perf_counter()
            s.step(steps)
            s.sync()
            el += time.perf_counter() - t0
            energies.append(s.energies().as_dict(lat.nfields))
    work = float(sum(lat.site_fields for lat in lattices)) * steps
    return EnsembleResult(el, work, energies)


# ---- serving --------------------------------------------------------------

@dataclass
class JobRecord:
    job_id: int
    site_field_updates: float
    arrival: float
    ready: float = -1.0       # host inputs generated
    admitted: float = -1.0    # joined the pool
    finished: float = -1.0    # last step done (seen at a block boundary)
    done: float = -1.0        # read back and retired
    energy: Optional[dict] = None
    status: str = "pending"

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def _percentile(xs: Sequence[float], q: float) -> float:
    return float(np.percentile(np.asarray(xs, np.float64), q)) if len(xs) else float("nan")


def summarize(records: Sequence[JobRecord], makespan: float) -> dict:
    ok = [r for r in records if r.status == "done"]
    lat = [r.latency for r in ok]
    return {
        "jobs": len(records), "completed": len(ok),
        "failed": sum(r.status == "failed" for r in records),
        "cancelled": sum(r.status == "cancelled" for r in records),
        "p50_latency_s": _percentile(lat, 50), "p99_latency_s": _percentile(lat, 99),
        "mean_latency_s": float(np.mean(lat)) if lat else float("nan"),
        "makespan_s": makespan,
        "site_field_updates_per_s": sum(r.site_field_updates for r in ok) / makespan,
        "breakdown_mean_s": {
            "host_init": float(np.mean([r.ready - r.arrival for r in ok])) if ok else float("nan"),
            "queue": float(np.mean([r.admitted - r.ready for r in ok])) if ok else float("nan"),
            "device": float(np.mean([r.finished - r.admitted for r in ok])) if ok else float("nan"),
            "readback": float(np.mean([r.done - r.finished for r in ok])) if ok else float("nan"),
        },
    }


class Server:
    """Continuous batching of simulation jobs on one GPU.

    Jobs arrive at their `arrival` times (seconds after start).  Inputs are
    generated by `workers` host threads from arrival on; ready jobs are
    admitted in arrival order while the budget allows; the pool then runs a
    block of steps sized to about `block_ms` of device time, after which
    finished members are read back and retired.  `cancel` drops a job from
    another thread while `run` serves.
    """

    def __init__(self, budget_bytes: int = 200 << 30, block_ms: float = 2.5,
                 workers: Optional[int] = None, precision: int = ce.CE_FP32,
                 read_fields: bool = False, pool_factory=None, make_inputs=None,
                 admit_threads: int = 4, short_first: bool = False, max_block_steps: int = 200,
                 rate_guess: float = 2e11, device_inputs: Optional[bool] = None):
        self.budget = budget_bytes
        self.block_ms = block_ms
        self.workers = workers or _host_workers()
        self.precision = precision
        self.read_fields = read_fields
        # injectable for testing the scheduling without a GPU
        self.pool_factory = pool_factory or (lambda budget: ce.Pool(budget))
        self.make_inputs = make_inputs or pinned_inputs
        # initial fields generated on the device at admission (the default
        # with the real pool and no host input generator given), or on host
        # threads from arrival on
        if device_inputs is None:
            device_inputs = pool_factory is None and make_inputs is None
        self.device_inputs = bool(device_inputs)
        # admissions in flight at once (each waits mostly on its upload and
        # start-up pass, so a few overlap well).  Short blocks (2.5 ms of
        # device time) let admissions and retirements in at frequent block
        # boundaries: against 20 ms blocks and 2 admission threads they cut
        # the median latency of the serving stream by 12% and the makespan
        # of 600 jobs released at once by 10% (measured, same GPU)
        self.admit_threads = max(1, int(admit_threads))
        # step budgets per block: shortest remaining work first (True) or
        # plain processor sharing, every member the same steps (False, the
        # default: the shortest-first run on the device is not yet validated)
        self.short_first = short_first
        self.max_block_steps = max_block_steps
        self.rate_guess = rate_guess   # site-field updates/s before any block was timed
        self.member_launch = (lambda lat: tuned_member_launch(lat, precision)) if pool_factory is None \
            else (lambda lat: None)
        self._cancel_lock = threading.Lock()
        self._cancel_req: List[int] = []
        self._serving = False
        # set by run(): the most device bytes the pool held, and the jobs
        # whose admission had to wait for memory
        self.peak_used_bytes = 0
        self.waited_for_memory = 0

    def cancel(self, job_id: int) -> bool:
        """Drop a job of the run in progress (thread-safe).

        A job not yet admitted is never admitted; a member of the pool is
        retired at the next block boundary, its fields not read back, and its
        memory goes back to the budget; a job already finished keeps its
        result.  The job's record gets status "cancelled".  Returns False,
        and records nothing, when no run is in progress."""
        with self._cancel_lock:
            if not self._serving:
                return False
            self._cancel_req.append(int(job_id))
            return True

    def _take_cancels(self) -> List[int]:
        with self._cancel_lock:
            req, self._cancel_req = self._cancel_req, []
        return req

    def _plan_block(self, pool, live, members, by_id, rate_est):
        """Steps of the next block and each member's budget in it.

        The block gets about block_ms of device time.  Plain processor
        sharing gives every member the same k steps.  Shortest-first hands
        the block's work to members in order of remaining work (site-fields
        x steps left), each up to its remaining steps, while every member
        keeps at least a quarter of its processor-sharing steps, so long jobs
        never stall.  Returns (k, site-field updates in the block)."""
        size = {pid: float(by_id[members[pid]].lattice.site_fields) for pid in live}
        left = {pid: pool.steps_left(pid) for pid in live}
        budget = self.block_ms * 1e-3 * rate_est
        k_ps = int(max(1, min(self.max_block_steps, budget / sum(size.values()))))
        if not self.short_first:
            return k_ps, sum(min(k_ps, left[p]) * size[p] for p in live)
        floor = max(1, k_ps // 4)
        q = {}
        for pid in sorted(live, key=lambda p: size[p] * left[p]):
            want = min(left[pid], self.max_block_steps)
            take = min(want, max(floor, int(budget // size[pid])))
            q[pid] = take
            budget -= take * size[pid]
        k = max(q.values())
        for pid in live:
            pool.set_quota(pid, q[pid] if q[pid] < min(left[pid], k) else -1)
        return k, sum(q[p] * size[p] for p in live)

    def run(self, jobs: Sequence[Job], progress=None) -> List[JobRecord]:
        """Serve `jobs`; progress(done, total), if given, is called as jobs
        finish (at most every 10 s)."""
        with self._cancel_lock:
            if self._serving:
                raise RuntimeError("Server.run is already serving")
            self._serving = True
            self._cancel_req = []
        try:
            return self._serve(jobs, progress)
        finally:
            with self._cancel_lock:
                self._serving = False
                self._cancel_req = []

    def _serve(self, jobs: Sequence[Job], progress) -> List[JobRecord]:
        recs = {j.job_id: JobRecord(j.job_id, float(j.lattice.site_fields) * j.lattice.steps,
                                    j.arrival) for j in jobs}
        pending = sorted(jobs, key=lambda j: j.arrival)
        by_id = {j.job_id: j for j in jobs}
        futures: Dict[int, cf.Future] = {}
        inputs: Dict[int, tuple] = {}
        members: Dict[int, int] = {}          # pool id -> job id
        ending: Dict[int, int] = {}           # pool id -> iteration its last step was enqueued
        adm_q: "queue.Queue" = queue.Queue()  # job ids with inputs, in arrival order
        adm_done: "queue.Queue" = queue.Queue()  # (pool id or None, job id, time)
        freed = threading.Condition()
        cancelled: set = set()                # job ids; read by the admission threads
        stop = -1
        rate_est = self.rate_guess            # site-field updates/s, refined as blocks run
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        nxt = 0
        ndone = 0
        last_note = [0.0]

        stopping = threading.Event()          # set when the run ends

        waited: set = set()                   # job ids that saw CE_EBUSY (admission threads)

        def admitter(pool):
            # Admissions run on these threads, beside the block loop: a job's
            # upload and start-up overlap the blocks in flight.  Jobs are taken
            # in arrival order; a job that does not fit the budget left waits
            # for a retirement, one larger than the whole budget fails.
            while True:
                jid = adm_q.get()
                if jid == stop:
                    return
                if jid in cancelled:
                    inputs.pop(jid, None)
                    continue
                lat = by_id[jid].lattice
                if not self.device_inputs:
                    phi, phid = inputs[jid][:2]
                cfg = self.member_launch(lat)
                while jid not in cancelled and not stopping.is_set():
                    try:
                        if self.device_inputs:
                            pid = pool.admit_generated(params_of(lat, self.precision), ce.lattice_init_spec(lat),
                                                       lat.steps, launch=cfg)
                        else:
                            pid = pool.admit(params_of(lat, self.precision), phi, phid, lat.steps, launch=cfg)
                        adm_done.put((pid, jid, now()))
                        break
                    except ce.CeError as e:
                        if e.status == ce.CE_EBUSY:
                            waited.add(jid)
                            with freed:
                                freed.wait(0.005)
                            continue
                        adm_done.put((None, jid, now()))
                        break
                inputs.pop(jid, None)

        def collect():
            nonlocal nxt
            # arrivals -> input generation; generated inputs -> admission queue
            while nxt < len(pending) and pending[nxt].arrival <= now():
                j = pending[nxt]
                if j.job_id in cancelled:
                    pass
                elif self.device_inputs:
                    # nothing to prepare on the host: straight to admission
                    recs[j.job_id].ready = now()
                    adm_q.put(j.job_id)
                else:
                    futures[j.job_id] = ex.submit(self.make_inputs, j.lattice)
                nxt += 1
            ready = sorted((k for k, f in futures.items() if f.done()), key=lambda k: (by_id[k].arrival, k))
            for jid in ready:
                if jid in cancelled:
                    futures.pop(jid)
                    continue
                inputs[jid] = futures.pop(jid).result()
                recs[jid].ready = now()
                adm_q.put(jid)

        if self.device_inputs or self.make_inputs is pinned_inputs:
            # create the GPU context here, before the input threads allocate
            # page-locked memory, rather than lazily inside one of them
            try:
                import torch
                if torch.cuda.is_available():
                    torch.cuda.init()
            except ImportError:
                pass
        with self.pool_factory(self.budget) as pool, cf.ThreadPoolExecutor(self.workers) as ex:
            threads = [threading.Thread(target=admitter, args=(pool,), daemon=True)
                       for _ in range(self.admit_threads)]
            for th in threads:
                th.start()
            try:
                # Pipelined: the next block is enqueued before the previous one
                # is waited for (the pool keeps at most two in flight), and a
                # member is retired one iteration after its last step was
                # enqueued, so the wait for its block overlaps the block
                # behind it.
                t_prev = None
                work_prev = 0.0
                it = 0
                while ndone < len(jobs):
                    it += 1
                    collect()
                    while True:
                        try:
                            pid, jid, t = adm_done.get_nowait()
                        except queue.Empty:
                            break
                        r = recs[jid]
                        if jid in cancelled:
                            # cancelled while its admission was under way
                            if pid is not None:
                                pool.retire(pid, read=False)
                                with freed:
                                    freed.notify_all()
                        elif pid is None:
                            r.status, r.done = "failed", t
                            ndone += 1
                        else:
                            members[pid] = jid
                            r.admitted, r.status = t, "running"
                            self.peak_used_bytes = max(self.peak_used_bytes, int(pool.info().used_bytes))
                    for jid in self._take_cancels():
                        r = recs.get(jid)
                        if r is None or r.status in ("done", "failed", "cancelled"):
                            continue
                        cancelled.add(jid)
                        r.status, r.done = "cancelled", now()
                        ndone += 1
                        pid = next((q for q, j in members.items() if j == jid), None)
                        if pid is not None:
                            # a member with steps still enqueued: retire waits
                            # for the pool's stream, then frees its memory
                            del members[pid]
                            ending.pop(pid, None)
                            pool.retire(pid, read=False)
                            with freed:
                                freed.notify_all()
                    live = [pid for pid in members if pid not in ending]
                    active_work = sum(float(by_id[members[pid]].lattice.site_fields) for pid in live)
                    if active_work > 0:
                        k, work = self._plan_block(pool, live, members, by_id, rate_est)
                        pool.run_block(k)
                        t = time.perf_counter()
                        if t_prev is not None and t - t_prev > 1e-4:
                            # one block ran per iteration in steady state
                            rate_est = 0.7 * rate_est + 0.3 * (work_prev / (t - t_prev))
                        t_prev, work_prev = t, work
                        for pid in live:
                            if pool.steps_left(pid) == 0:
                                ending[pid] = it
                    else:
                        t_prev = None
                    # members whose last block is not the newest one, or all
                    # of them once nothing more is enqueued
                    retire_now = [pid for pid, i in ending.items() if i < it or active_work == 0]
                    for pid in retire_now:
                        del ending[pid]
                        jid = members.pop(pid)
                        r = recs[jid]
                        try:
                            _, e = pool.poll(pid)
                            r.finished = now()
                            r.energy = e.as_dict(by_id[jid].lattice.nfields)
                            r.status = "done"
                        except ce.CeError:
                            r.finished = now()
                            r.status = "failed"
                        pool.retire(pid, read=self.read_fields)
                        r.done = now()
                        ndone += 1
                        if progress is not None and now() - last_note[0] >= 10.0:
                            last_note[0] = now()
                            progress(ndone, len(jobs))
                    if retire_now:
                        with freed:
                            freed.notify_all()
                    if active_work == 0 and not retire_now:
                        # nothing on the device: wait briefly for an admission
                        try:
                            item = adm_done.get(timeout=0.001)
                            adm_done.put(item)
                        except queue.Empty:
                            pass
            finally:
                # admission threads end before the pool is destroyed
                stopping.set()
                for _ in threads:
                    adm_q.put(stop)
                for th in threads:
                    th.join()
        self.waited_for_memory = len(waited)
        return [recs[j.job_id] for j in jobs]


def serve_sequential(jobs: Sequence[Job], workers: Optional[int] = None,
                     precision: int = ce.CE_FP32, device_inputs: bool = True, progress=None) -> List[JobRecord]:
    """First-come-first-served plain runs, one job on the GPU at a time; the
    initial fields are generated on the device (device_inputs) or on host
    threads ahead of time."""
    workers = workers or _host_workers()
    recs = [JobRecord(j.job_id, float(j.lattice.site_fields) * j.lattice.steps, j.arrival)
            for j in jobs]
    order = sorted(range(len(jobs)), key=lambda i: jobs[i].arrival)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    futures = {}
    last_note = [0.0]

    def generate(k):
        if device_inputs:
            recs[k].ready = now()
            return None
        out = lattice_initial(jobs[k].lattice, 1)
        recs[k].ready = now()
        return out

    with cf.ThreadPoolExecutor(workers) as ex:
        nxt = 0
        for i in order:
            j = jobs[i]
            while now() < j.arrival:
                # submit arrivals as they happen
                while nxt < len(order) and jobs[order[nxt]].arrival <= now():
                    k = order[nxt]
                    futures[k] = ex.submit(generate, k)
                    nxt += 1
                time.sleep(0.0005)
            while nxt < len(order) and jobs[order[nxt]].arrival <= now():
                k = order[nxt]
                futures[k] = ex.submit(generate, k)
                nxt += 1
            host = futures.pop(i).result()
            r = recs[i]
            r.admitted = now()
            lat = j.lattice
            try:
                with ce.Simulation.from_lattice(lat, precision) as s:
                    if host is None:
                        s.generate(ce.lattice_init_spec(lat))
                    else:
                        s.load(*host)
                    s.step(lat.steps)
                    r.energy = s.energies().as_dict(lat.nfields)
                    r.finished = now()
                r.status = "done"
            except ce.CeError:
                r.status = "failed"
            r.done = now()
            if progress is not None and now() - last_note[0] >= 10.0:
                last_note[0] = now()
                progress(sum(1 for x in recs if x.done >= 0), len(jobs))
    return recs
