"""The continuous-batching server on the GPU, end to end: jobs of the serving
stream arrive, are admitted with initial fields generated on the device, run
together in the pool and retire.  Each job's result must be bitwise the one
the same job gives run alone with the same launch, and cancelling a running
job must leave the others untouched."""
import threading

import pytest

from paper_0712_0813_amd import ce, serve
from paper_0712_0813_amd.workloads import Job, serving_mix

pytestmark = pytest.mark.gpu


def _small_jobs(n, steps_cap=300, spacing=0.02):
    """The first n jobs of the serving stream with 3-D N <= 64 or 2-D N = 256,
    capped at steps_cap steps, arriving every `spacing` seconds."""
    out = []
    for job in serving_mix(400):
        lat = job.lattice
        if (lat.dims == 3 and lat.N <= 64) or (lat.dims == 2 and lat.N == 256):
            out.append(Job(len(out), len(out) * spacing, lat.with_(steps=min(lat.steps, steps_cap))))
        if len(out) == n:
            break
    assert len(out) == n
    return out


def _alone(lat):
    """Final diagnostics of the job run as a lone simulation, with the launch
    the server gives it as a pool member."""
    cfg = serve.tuned_member_launch(lat) or ce.ce_pool_launch_for(serve.params_of(lat)).as_tuple()
    with ce.Simulation.from_lattice(lat) as s:
        s.set_launch(*cfg)
        s.generate(ce.lattice_init_spec(lat))
        s.step(lat.steps)
        return s.energies().as_dict(lat.nfields)


def test_server_results_equal_lone_runs_bitwise():
    jobs = _small_jobs(8)
    assert {j.lattice.dims for j in jobs} == {2, 3}
    recs = serve.Server(budget_bytes=8 << 30, block_ms=5.0).run(jobs)
    for j, r in zip(jobs, recs):
        print(j.job_id, j.lattice.dims, j.lattice.N, j.lattice.nfields, j.lattice.steps, r.status, flush=True)
        assert r.status == "done"
        assert r.energy["step"] == j.lattice.steps
        assert r.energy == _alone(j.lattice), j.job_id


def test_server_cancel_of_running_job_leaves_others_bitwise():
    jobs = _small_jobs(5)
    jobs[0] = Job(0, 0.0, jobs[0].lattice.with_(steps=10 ** 7))   # far longer than the test
    srv = serve.Server(budget_bytes=8 << 30, block_ms=5.0)
    timer = threading.Timer(2.0, srv.cancel, args=(0,))
    timer.start()
    recs = srv.run(jobs)
    timer.join()
    assert recs[0].status == "cancelled"
    assert recs[0].admitted >= 0            # it was running when cancelled
    for j, r in zip(jobs[1:], recs[1:]):
        assert r.status == "done"
        assert r.energy == _alone(j.lattice), j.job_id
