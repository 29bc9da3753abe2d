"""Achieved errors of the GPU path against the FP64 oracle, per result.

Not a test (pytest does not collect it): it runs the configurations' physics
on the GPU and in the oracle from the same seeded inputs and prints, as a
markdown table, the error actually reached for each result, beside the bar the
parity tests hold it to:

  - per site after 200 steps, for f and its half-step derivative: the parity
    metric max |g - o| / max(|o|, rms(o)), and max |g - o| over the rms of the
    fluctuation o - <o> (for a field near its background the first divides by
    ~1, the second by the ~1e-3 fluctuations);
  - per diagnostic (<f_i^2>, K_i, G_i, V, rho, a, a'), the worst relative
    error over every step of the run, and the worst absolute difference of
    the Friedmann residual;
  - for long runs, the same diagnostics sampled every 100 steps.

    python tests/achieved_errors.py [--long]
"""
import argparse
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import Oracle  # noqa: E402
from paper_0712_0813_amd import ce  # noqa: E402
from paper_0712_0813_amd.workloads import LATTICE32_STATIC as W0  # noqa: E402
from _parity import Case, energy_errors, run_pair, site_error  # noqa: E402

PER_SITE = [
    Case("lattice32_static (32^3, G=100, static)", W0.dims, W0.N, W0.nfields, W0.L, W0.dt, G=tuple(W0.G),
         seed=W0.seed),
    Case("lattice256_expanding physics (dx=20/256, dt=0.005, G=100) on 32^3", 3, 32, 2, 2.5, 0.005,
         G=(0.0, 100.0, 0.0), expansion=True),
    Case("lattice1024_expanding physics (dx=40/1024, dt=0.005, G=1000) on 48^3", 3, 48, 2, 48 * 40.0 / 1024, 0.005,
         G=(0.0, 1000.0, 0.0), expansion=True, seed=1),
]
LONG = [
    (Case("lattice256_expanding physics on 48^3, 2000 steps", 3, 48, 2, 48 * 20.0 / 256, 0.005, G=(0.0, 100.0, 0.0),
          expansion=True), 2000),
    (Case("lattice1024_expanding physics on 48^3, 500 steps", 3, 48, 2, 48 * 40.0 / 1024, 0.005, G=(0.0, 1000.0, 0.0),
          expansion=True, seed=1), 500),
]
PREC = {ce.CE_FP32: "FP32", ce.CE_FP64: "FP64"}


def fluct_error(g, o):
    d = o - o.mean()
    return float(np.max(np.abs(g - o)) / max(np.sqrt(np.mean(d * d)), 1e-300))


def diag_worst(log, olog, nf, expansion):
    worst = {}
    for g, o in zip(log, olog):
        for k, v in energy_errors(g, o, nf).items():
            worst[k] = max(worst.get(k, 0.0), v)
        if expansion:
            worst["resid(abs)"] = max(worst.get("resid(abs)", 0.0), abs(g["friedmann_residual"] - o.resid))
    return worst


def fmt(d, keys):
    return ", ".join(f"{k} {d[k]:.1e}" for k in keys if k in d)


def per_site_rows():
    rows = []
    for case in PER_SITE:
        for prec in (ce.CE_FP64, ce.CE_FP32):
            t0 = time.time()
            f, fd, log, orc = run_pair(case, prec, 200)
            parts = []
            for i in range(case.nfields):
                parts.append(f"f{i}: {site_error(f[i], orc.f[i]):.1e} / {fluct_error(f[i], orc.f[i]):.1e}")
                parts.append(f"f{i}': {site_error(fd[i], orc.pi[i]):.1e} / {fluct_error(fd[i], orc.pi[i]):.1e}")
            w = diag_worst(log, orc.log, case.nfields, case.expansion)
            keys = [f"mean_sq{i}" for i in range(case.nfields)] + [f"kin{i}" for i in range(case.nfields)] + \
                   [f"grad{i}" for i in range(case.nfields)] + ["pot", "rho", "a", "adot", "resid(abs)"]
            rows.append((case.name, PREC[prec], "; ".join(parts), fmt(w, keys)))
            print(f"[achieved] {case.name} {PREC[prec]} ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    return rows


def long_rows():
    rows = []
    for case, steps in LONG:
        t0 = time.time()
        phi, phid = case.inputs()

        def oracle_samples():
            orc = Oracle(case.oracle_params(), phi, phid)
            out = [orc.state]
            for _ in range(steps // 100):
                out.append(orc.step(100, record=False))
            return out

        with ThreadPoolExecutor(1) as ex:
            fut = ex.submit(oracle_samples)
            gpu = []
            with case.sim(ce.CE_FP32) as s:
                s.load(phi, phid)
                gpu.append(s.energies().as_dict(case.nfields))
                for _ in range(steps // 100):
                    s.step(100)
                    gpu.append(s.energies().as_dict(case.nfields))
            orc = fut.result()
        w = diag_worst(gpu, orc, case.nfields, case.expansion)
        end = energy_errors(gpu[-1], orc[-1], case.nfields)
        keys = [f"mean_sq{i}" for i in range(case.nfields)] + [f"kin{i}" for i in range(case.nfields)] + \
               [f"grad{i}" for i in range(case.nfields)] + ["pot", "rho", "a"]
        rows.append((case.name, "FP32", "every 100 steps: " + fmt(w, keys + ["resid(abs)"]),
                     "at the end: " + fmt(end, keys) +
                     f", resid {gpu[-1]['friedmann_residual']:.2e} (oracle {orc[-1].resid:.2e})"))
        print(f"[achieved] {case.name} ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    return rows


def translation_rows():
    """Shifted inputs against shifted outputs after 40 steps (the parity
    test's case): exact in real arithmetic."""
    case = PER_SITE[1]
    phi, phid = case.inputs()
    shift = (0, 5, 11, 3)
    rows = []
    for prec in (ce.CE_FP64, ce.CE_FP32):
        outs = []
        for sh in ((0, 0, 0, 0), shift):
            with case.sim(prec) as s:
                s.load(np.roll(phi, sh, axis=(0, 1, 2, 3)), np.roll(phid, sh, axis=(0, 1, 2, 3)))
                s.step(40)
                outs.append(s.read())
        parts = []
        for k, name in ((0, "f"), (1, "f'")):
            for i in range(case.nfields):
                a = np.roll(outs[0][k][i], shift[1:], axis=(0, 1, 2))
                b = outs[1][k][i]
                parts.append(f"{name}{i}: {site_error(b, a):.1e} / {fluct_error(b, a):.1e}")
        rows.append(("translation by (5, 11, 3), 40 steps, " + case.name, PREC[prec], "; ".join(parts), ""))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--long", action="store_true", help="also the long runs (volume averages)")
    args = ap.parse_args()
    rows = per_site_rows() + translation_rows()
    print("| run | storage | per site after 200 steps: parity metric / error over fluctuation rms | "
          "worst diagnostic error over all steps |")
    print("|---|---|---|---|")
    for r in rows:
        print("| " + " | ".join(r) + " |")
    if args.long:
        print()
        print("| run | storage | worst over the run | final step |")
        print("|---|---|---|---|")
        for r in long_rows():
            print("| " + " | ".join(r) + " |")


if __name__ == "__main__":
    main()
