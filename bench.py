"""Single-GPU throughput of the fused leapfrog step (site-field updates/s).

Workload: the 1024^3 two-field expanding lattice (lambda phi^4 + G phi^2 chi^2
with G = 1000, L = 40, dt = 0.005, FP32 fields with FP64 volume sums and a(t),
seed 1), seeded synthetic preheating-shaped initial conditions.  One "step" is
one leapfrog step of the whole lattice: drift, 7-point Laplacian, potential
derivative, kick, FP64 energy sums and the scale-factor update.

Prints one JSON line.  PyTorch supplies the device arena and the stream only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
PROFILE_JSON = os.path.join(ROOT, "profiles", "step3d_1024_counters.json")


# sources the 3-D step kernel is compiled from, and the build flags
KERNEL_SOURCES = ("paper_0712_0813_amd/csrc/ce_step3d.hip", "paper_0712_0813_amd/csrc/ce_device.hpp",
                  "paper_0712_0813_amd/csrc/ce_internal.hpp", "include/ce.h", "paper_0712_0813_amd/build.py")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(launch):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources with the same launch configuration; else None."""
    if not os.path.exists(PROFILE_JSON):
        return None
    with open(PROFILE_JSON) as fh:
        prof = json.load(fh)
    if prof.get("kernel_source_hash") != kernel_source_hash() or list(prof.get("launch", [])) != list(launch):
        return None
    return prof.get("hbm_bytes_per_launch")


STEP_KERNEL = "tiled3d_kernel<float, 2, 0, 0, 4, 64, 256>"


def _counter_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def counter_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, stats_csv, bench_log, out=PROFILE_JSON):
    """Per-launch HBM bytes of the 1024^3 step kernel from two rocprofv3 --pmc
    runs of this script (FETCH_SIZE, then WRITE_SIZE), scaled by what the same
    counters read for the 8 GiB copy of --copy-calibration (known bytes), with
    the kernel's average duration from a --kernel-trace --stats run and the
    launch tuple from the JSON line of the profiled run.  Writes `out`."""
    def per_dispatch(path, name):
        vals = {}
        for r in _counter_rows(path):
            if name(r["Kernel_Name"]):
                vals[int(r["Dispatch_Id"])] = vals.get(int(r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
        return [vals[k] for k in sorted(vals)]

    def is_step(n):
        return STEP_KERNEL + "(" in n

    def is_copy(n):
        return "__amd_rocclr_copyBuffer" in n

    copy_bytes = 8 * 1024 ** 3
    cf = max(per_dispatch(copy_fetch_csv, is_copy))
    cw = max(per_dispatch(copy_write_csv, is_copy))
    fetch_scale = copy_bytes / (cf * 1024)
    write_scale = copy_bytes / (cw * 1024)
    f = per_dispatch(fetch_csv, is_step)
    w = per_dispatch(write_csv, is_step)
    if len(f) < 4 or len(w) < 4:
        raise RuntimeError(f"too few step dispatches in the counter runs ({len(f)}, {len(w)})")
    fm, wm = sum(f[2:]) / len(f[2:]), sum(w[2:]) / len(w[2:])
    avg_ms = None
    for r in _counter_rows(stats_csv):
        if is_step(r["Name"]):
            avg_ms = float(r["AverageNs"]) / 1e6
    with open(bench_log) as fh:
        line = [ln for ln in fh if ln.startswith("{")][-1]
    launch = json.loads(line)["diagnostics"]["launch"]
    site_fields = 2 * 1024 ** 3
    prof = {"kernel": STEP_KERNEL, "workload": "lattice1024_expanding", "launch": launch,
            "kernel_source_hash": kernel_source_hash(), "dispatches": [len(f), len(w)],
            "fetch_size_kib": fm, "write_size_kib": wm, "fetch_scale": fetch_scale, "write_scale": write_scale,
            "hbm_read_bytes_per_launch": fm * 1024 * fetch_scale,
            "hbm_write_bytes_per_launch": wm * 1024 * write_scale,
            "hbm_bytes_per_launch": fm * 1024 * fetch_scale + wm * 1024 * write_scale,
            "reads_over_algorithmic": fm * 1024 * fetch_scale / (8.0 * site_fields),
            "writes_over_algorithmic": wm * 1024 * write_scale / (8.0 * site_fields),
            "kernel_avg_ms": avg_ms, "summary": "step3d_1024_lattice.md"}
    with open(out, "w") as fh:
        json.dump(prof, fh, indent=1)
        fh.write("\n")
    return prof


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        return None


def cpu_baseline(lat, threads=None, N=128, steps=80):
    """The FP64 oracle as it is, on a bounded sample of the workload: the same
    model, dx, dt and expansion on an N^3 periodic lattice for `steps` steps
    (about 12 s per run).  Timed once on one thread, then on every host core
    at once: `threads` independent copies of the lattice, one per thread (the
    oracle's C loop releases the interpreter lock).  `value` is the all-core
    rate."""
    import concurrent.futures as cf
    from oracle import Oracle, OracleParams
    from paper_0712_0813_amd.inputs import make_initial

    threads = threads or os.cpu_count() or 1
    L = lat.L * N / lat.N
    p = OracleParams(dims=lat.dims, N=N, nfields=lat.nfields, L=L, dt=lat.dt, lam=lat.lam,
                     G=lat.G, mu2=lat.mu2, expansion=lat.expansion, kappa=lat.kappa)
    phi, phid = make_initial(lat.seed, lat.dims, N, L, lat.nfields, lat.m_eff2(), amp=lat.amp)
    per_run = float(N ** lat.dims * lat.nfields * steps)

    orc = Oracle(p, phi, phid)
    t0 = time.perf_counter()
    orc.step(steps, record=False)
    el1 = time.perf_counter() - t0
    print(f"[bench] cpu baseline, 1 thread: {el1:.1f} s", file=sys.stderr, flush=True)

    copies = [Oracle(p, phi, phid) for _ in range(threads)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda o: o.step(steps, record=False), copies))
    eln = time.perf_counter() - t0
    # every copy ran the same arithmetic on the same input
    assert all(np.array_equal(o.f, orc.f) for o in copies)
    print(f"[bench] cpu baseline, {threads} threads: {eln:.1f} s", file=sys.stderr, flush=True)
    return {"value": threads * per_run / eln, "unit": "site-field updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{N}^3 x {lat.nfields} fields, same model/dx/dt/expansion, {steps} steps, FP64; "
                      f"{threads} independent copies on {threads} threads in {eln:.1f} s",
            "cpu_model": host_cpu_model(),
            "single_thread": {"value": per_run / el1, "seconds": el1}}


def ensemble_section(count: int, steps: int) -> dict:
    """`count` independent 64^3 two-field lattices advanced together (one
    launch per class per step, graph-captured blocks) against the same
    lattices run one after another as plain simulations."""
    from paper_0712_0813_amd import serve
    from paper_0712_0813_amd.workloads import ensemble_512x64
    lats = ensemble_512x64(count=count, steps=steps)
    t0 = time.perf_counter()
    inputs = serve.generate_all(lats)
    gen = time.perf_counter() - t0
    print(f"[bench] ensemble inputs: {count} lattices in {gen:.1f} s", file=sys.stderr, flush=True)
    bat = serve.run_batched(lats, inputs, steps, block=50)
    print(f"[bench] ensemble batched: {bat.seconds:.2f} s", file=sys.stderr, flush=True)
    seq = serve.run_sequential(lats, inputs, steps)
    print(f"[bench] ensemble sequential: {seq.seconds:.2f} s", file=sys.stderr, flush=True)
    worst = {}
    for k in ("a", "rho", "pot"):
        worst[k] = max(abs(x[k] - y[k]) / max(abs(y[k]), 1e-300) for x, y in zip(bat.energies, seq.energies))
    worst["mean_sq"] = max(abs(x["mean_sq"][i] - y["mean_sq"][i]) / max(abs(y["mean_sq"][i]), 1e-300)
                           for x, y in zip(bat.energies, seq.energies) for i in range(2))
    return {"workload": "ensemble_512x64", "lattices": count, "steps": steps,
            "batched_site_field_updates_per_s": bat.rate,
            "sequential_site_field_updates_per_s": seq.rate,
            "speedup_vs_sequential": bat.rate / seq.rate,
            "batched_seconds": bat.seconds, "sequential_seconds": seq.seconds,
            "max_rel_diff_batched_vs_sequential": worst}


def serving_section(njobs: int) -> dict:
    """The first `njobs` jobs of the Poisson serving stream, replayed in real
    time: continuous batching under a 200 GB budget against first-come
    first-served plain runs of the same jobs."""
    from paper_0712_0813_amd import serve
    from paper_0712_0813_amd.workloads import serving_mix
    jobs = serving_mix(2000)[:njobs]
    note = lambda done, total: print(f"[bench] serving: {done}/{total} jobs done", file=sys.stderr, flush=True)
    srv = serve.Server(budget_bytes=200 << 30)
    recs = srv.run(jobs, progress=note)
    cb = serve.summarize(recs, max(r.done for r in recs))
    print(f"[bench] serving continuous batching: p50 {cb['p50_latency_s']:.2f} s, "
          f"p99 {cb['p99_latency_s']:.2f} s", file=sys.stderr, flush=True)
    srecs = serve.serve_sequential(jobs, progress=note)
    sq = serve.summarize(srecs, max(r.done for r in srecs))
    print(f"[bench] serving sequential: p50 {sq['p50_latency_s']:.2f} s, "
          f"p99 {sq['p99_latency_s']:.2f} s", file=sys.stderr, flush=True)
    return {"workload": "serving_mix", "jobs": njobs, "of_stream": 2000, "arrival_rate_per_s": 20.0,
            "initial_fields": "generated on the device at admission",
            "budget_bytes": 200 << 30, "continuous_batching": cb, "sequential_fcfs": sq}


def serving_capacity_section(njobs: int, tight_budget_gb: int = 16) -> dict:
    """The first `njobs` jobs of the serving stream released together at t = 0:
    capacity (site-field updates over the makespan) of continuous batching
    against first-come first-served plain runs, and continuous batching under
    a budget small enough that admission by memory binds."""
    from paper_0712_0813_amd import serve
    from paper_0712_0813_amd.workloads import Job, serving_mix
    jobs = [Job(j.job_id, 0.0, j.lattice) for j in serving_mix(2000)[:njobs]]
    note = lambda done, total: print(f"[bench] capacity: {done}/{total} jobs done", file=sys.stderr, flush=True)
    out = {"workload": "serving_mix, released at t = 0", "jobs": njobs, "of_stream": 2000,
           "offered_site_field_updates": float(sum(j.lattice.site_fields * j.lattice.steps for j in jobs))}
    srv = serve.Server(budget_bytes=200 << 30)
    recs = srv.run(jobs, progress=note)
    out["continuous_batching"] = serve.summarize(recs, max(r.done for r in recs))
    out["continuous_batching"]["peak_used_bytes"] = srv.peak_used_bytes
    print(f"[bench] capacity, continuous batching: {out['continuous_batching']['makespan_s']:.1f} s",
          file=sys.stderr, flush=True)
    srecs = serve.serve_sequential(jobs, progress=note)
    out["sequential_fcfs"] = serve.summarize(srecs, max(r.done for r in srecs))
    print(f"[bench] capacity, sequential: {out['sequential_fcfs']['makespan_s']:.1f} s", file=sys.stderr,
          flush=True)
    out["capacity_ratio"] = (out["continuous_batching"]["site_field_updates_per_s"] /
                             out["sequential_fcfs"]["site_field_updates_per_s"])
    tight = serve.Server(budget_bytes=tight_budget_gb << 30)
    trecs = tight.run(jobs, progress=note)
    t = serve.summarize(trecs, max(r.done for r in trecs))
    t.update({"budget_bytes": tight_budget_gb << 30, "peak_used_bytes": tight.peak_used_bytes,
              "jobs_that_waited_for_memory": tight.waited_for_memory})
    out["continuous_batching_tight_budget"] = t
    print(f"[bench] capacity, {tight_budget_gb} GB budget: {t['makespan_s']:.1f} s, "
          f"{tight.waited_for_memory} jobs waited for memory", file=sys.stderr, flush=True)
    return out


def device_copy_rate(torch, gib: int = 4) -> float:
    """Read+write GB/s of a plain device-to-device copy of `gib` GiB."""
    n = gib * 1024 ** 3 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del x, y
    torch.cuda.empty_cache()
    return 8.0 * n / (ms / 1e3) / 1e9


def host_io_section(ce, np, lat, steps: int) -> dict:
    """One whole job through host memory: FP64 fields loaded from pageable host
    arrays, `steps` steps, both arrays of every field read back as FP64.  The
    input is the workload's seeded field generated at 32^3 and tiled to the
    full lattice (same size, physics and per-site values as any 32^3-periodic
    input), which keeps the host-side generation short.  Reports the job's
    rate including the host transfers beside its device-only rate."""
    from paper_0712_0813_amd.inputs import make_initial
    base = 32
    reps = (1,) + (lat.N // base,) * lat.dims
    phi, phid = make_initial(lat.seed, lat.dims, base, lat.L * base / lat.N, lat.nfields, lat.m_eff2(), lat.amp,
                             lat.background)
    big_phi, big_phid = np.tile(phi, reps), np.tile(phid, reps)
    with ce.Simulation.from_lattice(lat) as s:
        s.sync()
        t0 = time.perf_counter()
        s.load(big_phi, big_phid)
        s.sync()
        t1 = time.perf_counter()
        s.step(steps)
        s.sync()
        t2 = time.perf_counter()
        f, fd = s.read()
        t3 = time.perf_counter()
    upd = float(lat.N ** lat.dims * lat.nfields * steps)
    print(f"[bench] host io: load {t1 - t0:.2f} s, steps {t2 - t1:.2f} s, readback {t3 - t2:.2f} s",
          file=sys.stderr, flush=True)
    return {"steps": steps, "input": "seeded 32^3 field tiled to the lattice, FP64 host arrays",
            "load_s": t1 - t0, "load_GBps": (big_phi.nbytes + big_phid.nbytes) / (t1 - t0) / 1e9,
            "step_s": t2 - t1, "readback_s": t3 - t2, "readback_GBps": (f.nbytes + fd.nbytes) / (t3 - t2) / 1e9,
            "device_updates_per_s": upd / (t2 - t1), "pcie_inclusive_updates_per_s": upd / (t3 - t0)}


def image_section(ce, np, sim) -> dict:
    """Grid image of the 1024^3 state: save into a fresh (pageable) host
    buffer, then restore into the same simulation; rates over the image size."""
    n = ce.ce_image_bytes(sim)
    buf = np.empty(n, np.uint8)
    t0 = time.perf_counter()
    ce.ce_save_image(sim, buf)
    t_save = time.perf_counter() - t0
    t0 = time.perf_counter()
    ce.ce_save_image(sim, buf)          # again, into pages already touched
    t_save2 = time.perf_counter() - t0
    step = ce.ce_get_step(sim)
    t0 = time.perf_counter()
    ce.ce_restore_image(sim, buf)
    t_restore = time.perf_counter() - t0
    assert ce.ce_get_step(sim) == step
    del buf
    gb = n / 1e9
    return {"image_GB": gb, "save_s": t_save, "save_GBps": gb / t_save, "save_touched_GBps": gb / t_save2,
            "restore_s": t_restore, "restore_GBps": gb / t_restore}


def step_block_section(ce) -> dict:
    """Per-step time of small lattices (3-D, 2 fields, expanding) with plain
    launches against captured step blocks of 32 (HIP events on the
    simulation's stream, 1024 steps each)."""
    out = {}
    for N in (32, 64, 128):
        params = ce.make_params(3, N, 2, 10.0 * N / 64, 0.01, G=(0.0, 100.0, 0.0), expansion=True,
                                kappa=2.94)
        sim = ce.ce_create(params)
        try:
            ce.ce_generate_fields(sim, ce.make_init_spec(N, [3.0, 100.0]))
            row = {}
            for sb in (0, 32):
                ce.ce_set_step_block(sim, sb)
                ce.ce_time_steps(sim, 64)     # warm-up, builds the graph
                row["plain_ms" if sb == 0 else "graph32_ms"] = ce.ce_time_steps(sim, 1024) / 1024
            row["speedup"] = row["plain_ms"] / row["graph32_ms"]
            out[f"{N}^3"] = row
        finally:
            ce.ce_destroy(sim)
    return out


def lattice256_section(ce) -> dict:
    """The 256^3 expanding workload at its full length (2000 steps), lone,
    with the tuned launch when the cache holds one for the current sources
    (else the default): per-step time and algorithmic GB/s."""
    from paper_0712_0813_amd import autotune
    from paper_0712_0813_amd.workloads import LATTICE256_EXPANDING as W
    tuned = autotune.lookup(W.dims, W.N, W.nfields, ce.CE_FP32)
    with ce.Simulation.from_lattice(W, precision=ce.CE_FP32) as s:
        s.generate(ce.lattice_init_spec(W))
        if tuned:
            s.set_launch(*tuned)
        s.time_steps(64)
        ms = s.time_steps(W.steps)
        e = s.energies()
        launch = list(s.get_launch().as_tuple())
    per = ms / W.steps
    return {"workload": W.name, "steps": W.steps, "ms_per_step": per,
            "site_field_updates_per_s": W.site_fields / (per / 1e3),
            "algorithmic_GBps": 16.0 * W.site_fields / (per / 1e3) / 1e9, "launch": launch,
            "launch_source": "tuning cache (same source hash)" if tuned else "library default",
            "final_a": e.a, "friedmann_residual": e.friedmann_residual}


def lattice2d_section(ce, N: int = 4096, steps: int = 500) -> dict:
    """The 2-D streaming pass on an N^2 two-field lattice with the 1024^3
    workload's physics (grid spacing, time step, coupling, expansion), lone,
    default launch, seeded host-generated inputs: per-step time and
    algorithmic GB/s."""
    from paper_0712_0813_amd.inputs import make_initial
    from paper_0712_0813_amd.workloads import LATTICE1024_EXPANDING as W
    lat = W.with_(name=f"lattice{N}sq_expanding", dims=2, N=N, L=W.dx * N)
    phi, phid = make_initial(lat.seed, 2, N, lat.L, lat.nfields, lat.m_eff2(), amp=lat.amp,
                             background=lat.background)
    with ce.Simulation.from_lattice(lat, precision=ce.CE_FP32) as s:
        s.load(phi, phid)
        del phi, phid
        s.time_steps(64)
        ms = s.time_steps(steps)
        launch = list(s.get_launch().as_tuple())
    per = ms / steps
    gbs = 16.0 * lat.site_fields / (per / 1e3) / 1e9
    return {"workload": lat.name, "dims": 2, "N": N, "nfields": lat.nfields, "steps": steps, "ms_per_step": per,
            "site_field_updates_per_s": lat.site_fields / (per / 1e3), "algorithmic_GBps": gbs,
            "frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "launch": launch}


def spectrum_section(ce, np, sim, nfields: int) -> dict:
    """Radially binned spectra of every field (field and derivative) of the
    1024^3 state, timed on the host around each synchronous call."""
    out = {"seconds_per_field": [], "bins": ce.ce_spectrum_bins(sim)}
    for i in range(nfields):
        t0 = time.perf_counter()
        pf, pd, cnt = ce.ce_spectrum(sim, i)
        out["seconds_per_field"].append(time.perf_counter() - t0)
        out.setdefault("parseval_sum_f", []).append(float(pf.sum()))
    return out


def run_info_of(torch, dev) -> dict:
    """GPU, architecture, host core count and source revision of the run."""
    props = torch.cuda.get_device_properties(dev)
    rev = None
    try:
        rev = subprocess.run(["git", "-C", ROOT, "rev-parse", "--short", "HEAD"], capture_output=True,
                             text=True, timeout=10).stdout.strip() or None
    except (OSError, subprocess.SubprocessError):
        pass
    cpu = host_cpu_model()
    return {"gpu": props.name, "arch": getattr(props, "gcnArchName", None),
            "compute_units": props.multi_processor_count, "hbm_GiB": round(props.total_memory / 2 ** 30, 1),
            "host_cpu": cpu, "host_cores": os.cpu_count(), "torch": torch.__version__, "hip": torch.version.hip,
            "git_rev": rev}


def copy_calibration(torch):
    """A plain device copy of 8 GiB (reads 8 GiB, writes 8 GiB), the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    n = 2 * 1024 ** 3
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": ms,
                      "GBps_read_plus_write": 8 * n / (ms / 1e3) / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--step-block", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--N", type=int, default=None, help="override the lattice edge (testing only)")
    ap.add_argument("--ensemble", type=int, default=512,
                    help="lattices of the 64^3 ensemble (0 skips the ensemble section)")
    ap.add_argument("--ensemble-steps", type=int, default=1000)
    ap.add_argument("--serve-jobs", type=int, default=2000,
                    help="jobs of the 2000-job serving stream replayed in real time, about 100 s per "
                         "policy for all of them (0 skips the serving section)")
    ap.add_argument("--capacity-jobs", type=int, default=600,
                    help="jobs of the serving stream released together for the capacity and tight-budget "
                         "runs (0 skips them)")
    ap.add_argument("--no-image", action="store_true", help="skip the grid-image save/restore timing")
    ap.add_argument("--host-io", action="store_true",
                    help="also time one whole job loaded from and read back to host memory (PCIe-inclusive rate)")
    ap.add_argument("--tune", action="store_true",
                    help="time every launch candidate for the workload first and run with the fastest")
    ap.add_argument("--counter-summary", nargs=6, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV",
                                                             "STATS_CSV", "BENCH_LOG"),
                    help="write the step kernel's per-launch HBM traffic from rocprofv3 outputs (no GPU)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 8 GiB device copy (known bytes) for counter calibration")
    args = ap.parse_args()
    if args.counter_summary:
        print(json.dumps(counter_summary(*args.counter_summary), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_0712_0813_amd import ce
    from paper_0712_0813_amd.workloads import LATTICE1024_EXPANDING

    from paper_0712_0813_amd import autotune
    lat = LATTICE1024_EXPANDING
    if args.N:
        lat = lat.with_(N=args.N, L=lat.L * args.N / lat.N)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    run_info = run_info_of(torch, dev)
    # launch configuration: tuned now (--tune), else a cached choice measured
    # on the current kernel sources, else the library's default
    if args.tune:
        t_tune = time.perf_counter()
        tuned = autotune.tune(lat.dims, lat.N, lat.nfields, ce.CE_FP32)
        tuned["tune_s"] = time.perf_counter() - t_tune
        launch_source = "tuned in this run"
        print(f"[bench] tuned in {tuned['tune_s']:.1f} s: {tuned['launch']}", file=sys.stderr, flush=True)
    else:
        tuned = autotune.lookup_entry(lat.dims, lat.N, lat.nfields, ce.CE_FP32)
        launch_source = "tuning cache (same source hash)" if tuned else "library default"
    stream = torch.cuda.Stream(device=dev)
    params = ce.make_params(lat.dims, lat.N, lat.nfields, lat.L, lat.dt, lam=lat.lam, G=lat.G,
                            mu2=lat.mu2, expansion=lat.expansion, kappa=lat.kappa,
                            precision=ce.CE_FP32, stream=stream.cuda_stream)
    nbytes = ce.ce_required_bytes(params)
    arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = arena.data_ptr()
    params.arena = (base + 255) // 256 * 256
    params.arena_bytes = nbytes

    sim = ce.ce_create(params)
    # seeded initial fields generated on the device (untimed; the start-up
    # half step runs with them)
    t_init = time.perf_counter()
    ce.ce_generate_fields(sim, ce.lattice_init_spec(lat))
    ce.ce_sync(sim)
    t_init = time.perf_counter() - t_init
    print(f"[bench] fields generated on the device ({t_init:.2f} s)", file=sys.stderr, flush=True)
    if tuned:
        ce.ce_set_launch(sim, *tuned["launch"])
    ce.ce_set_step_block(sim, args.step_block)

    # warmup covers at least one whole step block, so the captured graph is
    # built before the timed region (reported as warmup_requested / warmup)
    warmup_requested = args.warmup
    if args.step_block > 0 and args.warmup < args.step_block:
        args.warmup = args.step_block
    ce.ce_step(sim, args.warmup)
    ce.ce_sync(sim)
    print(f"[bench] warmup {args.warmup} steps done", file=sys.stderr, flush=True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    ce.ce_step(sim, args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    e = ce.ce_energies(sim)
    launch = list(ce.ce_get_launch(sim).as_tuple())
    spectra = spectrum_section(ce, np, sim, lat.nfields)
    image = None if args.no_image else image_section(ce, np, sim)
    ce.ce_destroy(sim)
    del arena
    torch.cuda.empty_cache()
    host_io = host_io_section(ce, np, lat, args.steps) if args.host_io else None
    copy_gbs = device_copy_rate(torch)
    from paper_0712_0813_amd import ceiling as ceiling_probe
    ceiling = ceiling_probe.measure(torch)

    site_fields = lat.N ** lat.dims * lat.nfields
    ms_per_step = ms / args.steps
    value = site_fields * args.steps / (ms / 1e3)
    alg_bytes = 16.0 * site_fields  # read d, p; write d, p (FP32)
    achieved = alg_bytes / (ms_per_step / 1e3) / 1e9
    traffic = measured_traffic(launch)
    out = {
        "metric": "site-field updates/s + % HBM roofline (1024^3); ensemble p50/p99 job latency",
        "value": value,
        "unit": "site-field updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_requested": warmup_requested,
        "warmup_note": (f"raised to one whole step block ({args.step_block} steps) so the captured graph "
                        "is built before the timed region") if args.warmup != warmup_requested else None,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": lat.name, "dims": lat.dims, "N": lat.N, "nfields": lat.nfields,
                   "G": lat.G[1], "L": lat.L, "dt": lat.dt, "expansion": lat.expansion,
                   "seed": lat.seed, "sums_and_scale_factor": "f64",
                   "initial_fields": "seeded Gaussian random fields generated on the device",
                   "step_block": args.step_block, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "diagnostics": {"step": int(e.step), "a": e.a, "rho": e.rho,
                        "friedmann_residual": e.friedmann_residual, "init_s": t_init, "run_info": run_info,
                        "launch": launch,
                        "launch_source": launch_source,
                        "source_hash": autotune.source_hash(),
                        "tuned": tuned,
                        # rates the memory system reaches on the same GPU: a
                        # plain device copy, and the best read+write copy,
                        # read-only and write-only streams of the probe sweep
                        "device_copy_GBps": copy_gbs,
                        "frac_of_device_copy": achieved / copy_gbs,
                        "stream_ceiling": ceiling,
                        "frac_of_copy_ceiling": achieved / ceiling["copy"]["GBps"],
                        # HBM bytes the counters count per launch, over the launch time
                        "counter_traffic_GBps": (traffic / (ms_per_step / 1e3) / 1e9) if traffic else None},
    }
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)
    out["spectra"] = spectra
    if image is not None:
        out["image"] = image
    if host_io is not None:
        out["host_io"] = host_io
    out["step_blocks"] = step_block_section(ce)
    out["lattice256"] = lattice256_section(ce)
    out["lattice2d"] = lattice2d_section(ce)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lat)
    if args.ensemble > 0:
        out["ensemble"] = ensemble_section(args.ensemble, args.ensemble_steps)
    if args.serve_jobs > 0:
        out["serving"] = serving_section(args.serve_jobs)
    if args.capacity_jobs > 0:
        out["serving_capacity"] = serving_capacity_section(args.capacity_jobs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
