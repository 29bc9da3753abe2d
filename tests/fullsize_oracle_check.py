"""The 1024^3 benchmark lattice itself against the oracle, at full size.

Not a test (pytest does not collect it): it needs about 90 GB of host memory
and several minutes of one host core per step.  Both sides start from the
benchmark's own initial conditions (seed 1, the 1024^3 two-field expanding
workload): the GPU generates them on the device as `bench.py` does; the
oracle builds the same fields from its own generator's modes (`oracle.grf_modes`,
placed at n mod N and summed by one inverse FFT, as `oracle.grf_field` does,
with SciPy's multi-threaded FFT for speed).  Both then take the start-up
half step and `--steps` leapfrog steps, the GPU in the benchmark's launch
(the tuned one when the cache holds it).  Printed: every step's volume
averages (<f_i>, <f_i^2>, K_i, G_i, V, rho, a, a') as relative errors against
the oracle, and per-site errors of f and its derivative at sampled sites
after the last step (the parity metric and the error over the fluctuation
rms).

    python tests/fullsize_oracle_check.py [--steps 2] [--sites 200000]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

import oracle as orc_mod  # noqa: E402
from oracle import Oracle, OracleParams  # noqa: E402
from oracle.oracle import FIELD, MOMENTUM  # noqa: E402
from paper_0712_0813_amd import autotune, ce  # noqa: E402
from paper_0712_0813_amd.workloads import LATTICE1024_EXPANDING as W  # noqa: E402
from _parity import energy_errors  # noqa: E402

T0 = time.time()


def note(msg):
    print(f"[fullsize-oracle {time.time() - T0:7.1f} s] {msg}", flush=True)


def oracle_field(field, kind, meff2, W=W):
    """delta(x) of one array from the oracle generator's modes (the sum
    oracle.grf_field forms), transformed with SciPy's FFT on every core."""
    import scipy.fft
    c = orc_mod.grf_modes(W.seed, field, kind, 3, W.N, W.L, W.amp, meff2)
    K = W.N // 4
    full = np.zeros((W.N,) * 3, np.complex128)
    idx = np.arange(-K, K + 1) % W.N
    full[np.ix_(idx, idx, idx)] = c
    del c
    out = scipy.fft.ifftn(full, overwrite_x=True, workers=os.cpu_count())
    del full
    return np.ascontiguousarray(out.real) * float(W.N) ** 3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--sites", type=int, default=200000)
    args = ap.parse_args()
    S = args.steps
    sites = np.random.default_rng(11).integers(0, W.N ** 3, args.sites)

    # GPU: the benchmark's lattice, its launch, S steps
    with ce.Simulation.from_lattice(W, precision=ce.CE_FP32) as s:
        tuned = autotune.lookup(W.dims, W.N, W.nfields, ce.CE_FP32)
        if tuned:
            s.set_launch(*tuned)
        s.generate(ce.lattice_init_spec(W))
        s.set_step_block(0)
        s.step(S)
        launch = s.get_launch().as_tuple()
        log = [e.as_dict(W.nfields) for e in s.energy_log(S + 1)]
        got = [s.read_sites(i, sites) for i in range(W.nfields)]
    note(f"GPU: {S} steps with launch {launch}")

    # oracle: the same initial conditions from its own generator
    meff = W.m_eff2()
    shape = (W.nfields,) + (W.N,) * 3
    phi = np.empty(shape, np.float64)
    phid = np.empty(shape, np.float64)
    for i in range(W.nfields):
        phi[i] = oracle_field(i, FIELD, meff[i]) + W.background[i]
        note(f"oracle field {i} generated")
        phid[i] = oracle_field(i, MOMENTUM, meff[i])
        note(f"oracle derivative {i} generated")
    p = OracleParams(dims=3, N=W.N, nfields=W.nfields, L=W.L, dt=W.dt, lam=W.lam, G=tuple(W.G),
                     mu2=tuple(W.mu2), expansion=W.expansion, kappa=W.kappa)
    orc = Oracle(p, phi, phid)
    del phi, phid
    note("oracle start-up done")
    for k in range(S):
        orc.step(1)
        note(f"oracle step {k + 1} done")

    print("\n| step | worst volume-average errors (relative; residual absolute) |")
    print("|---|---|")
    for g, o in zip(log, orc.log):
        errs = energy_errors(g, o, W.nfields)
        keys = ["mean0", "mean1", "mean_sq0", "mean_sq1", "kin0", "kin1", "grad0", "grad1", "pot", "rho", "a",
                "adot"]
        txt = ", ".join(f"{k} {errs[k]:.1e}" for k in keys if k in errs)
        txt += f", residual {abs(g['friedmann_residual'] - o.resid):.1e}"
        print(f"| {g['step']} | {txt} |")
    print(f"\n| array (after {S} steps, {args.sites} sampled sites) | parity metric | over fluctuation rms |")
    print("|---|---|---|")
    for i in range(W.nfields):
        for name, g, o in ((f"f{i}", got[i][0], orc.f[i].ravel()[sites]),
                           (f"f{i}'", got[i][1], orc.pi[i].ravel()[sites])):
            full = orc.f[i] if name == f"f{i}" else orc.pi[i]
            rms = float(np.sqrt(np.mean(full * full)))
            flu = float(np.std(full))
            err = np.abs(g - o)
            print(f"| {name} | {np.max(err / np.maximum(np.abs(o), rms)):.1e} | {np.max(err) / flu:.1e} |")
    note("done")


if __name__ == "__main__":
    main()
