"""Shared helpers for GPU-vs-oracle parity tests."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

from oracle import Oracle, OracleParams
from paper_0712_0813_amd import ce
from paper_0712_0813_amd.inputs import make_initial
from paper_0712_0813_amd.workloads import DEFAULT_KAPPA

# per-site tolerances after 200 steps (relative, floored by the field's rms)
TOL_SITE = {ce.CE_FP64: 1e-12, ce.CE_FP32: 1e-4}
# volume means, energies and a(t)
TOL_MEAN = {ce.CE_FP64: 1e-11, ce.CE_FP32: 1e-4}


@dataclass(frozen=True)
class Case:
    name: str
    dims: int
    N: int
    nfields: int
    L: float
    dt: float
    G: Tuple[float, ...] = (0.0, 0.0, 0.0)
    mu2: Tuple[float, ...] = (0.0, 0.0, 0.0)
    lam: float = 1.0
    expansion: bool = False
    kappa: float = DEFAULT_KAPPA
    seed: int = 0
    amp: float = 1e-3
    vacuum: float = 0.0
    background: Tuple[float, ...] = (1.0, 0.0, 0.0)
    # user-defined polynomial potential ((coef, (e0, e1, e2)), ...); empty:
    # the quartic model with lam, G, mu2, vacuum
    terms: Tuple = ()

    def m_eff2(self):
        """Curvature of the potential at the background, floored at 0 (only
        shapes the initial spectrum; tachyonic bands get omega = k)."""
        b0 = self.background[0]
        out = [max(0.0, 3.0 * self.lam * b0 * b0 + self.mu2[0])]
        for j in range(1, self.nfields):
            out.append(max(0.0, self.G[j] * b0 * b0 + self.mu2[j]))
        return out

    def oracle_params(self) -> OracleParams:
        return OracleParams(dims=self.dims, N=self.N, nfields=self.nfields, L=self.L, dt=self.dt,
                            lam=self.lam, G=self.G, mu2=self.mu2, expansion=self.expansion,
                            kappa=self.kappa, vacuum=self.vacuum, terms=list(self.terms) or None)

    def inputs(self):
        return make_initial(self.seed, self.dims, self.N, self.L, self.nfields, self.m_eff2(),
                            amp=self.amp, background=self.background)

    def sim(self, precision: int, **kw) -> ce.Simulation:
        return ce.Simulation(self.dims, self.N, self.nfields, self.L, self.dt, lam=self.lam, G=self.G,
                             mu2=self.mu2, expansion=self.expansion, kappa=self.kappa, vacuum=self.vacuum,
                             precision=precision, terms=list(self.terms) or None, **kw)

    def params(self, precision: int = ce.CE_FP32) -> ce.ce_params:
        return ce.make_params(self.dims, self.N, self.nfields, self.L, self.dt, lam=self.lam, G=self.G,
                              mu2=self.mu2, expansion=self.expansion, kappa=self.kappa, vacuum=self.vacuum,
                              precision=precision, terms=list(self.terms) or None)


def rounded(x: np.ndarray, precision: int) -> np.ndarray:
    """Oracle inputs for a run in `precision`.  The GPU keeps each field as an
    FP64 homogeneous reference plus a deviation in the storage type, so its
    initial state equals the FP64 input to better than 1e-7 of the deviations;
    the oracle therefore starts from the unrounded inputs and the comparison
    measures the whole error, representation included."""
    return x.copy()


def site_error(g: np.ndarray, o: np.ndarray) -> float:
    """max_x |g - o| / max(|o(x)|, rms(o)) for one field's array."""
    rms = np.sqrt(np.mean(o * o))
    den = np.maximum(np.abs(o), rms if rms > 0 else 1e-300)
    return float(np.max(np.abs(g - o) / den))


ENERGY_KEYS = ("a", "adot", "rho", "pot")
FIELD_KEYS = ("kin", "grad", "mean_sq")


def energy_errors(g: dict, o, nf: int) -> Dict[str, float]:
    """Relative errors of the diagnostics of one step (GPU dict vs oracle state)."""
    out = {}
    for k in ENERGY_KEYS:
        ov = getattr(o, k)
        gv = g[k]
        scale = abs(ov) if ov != 0 else 1.0
        out[k] = abs(gv - ov) / scale
    rho = abs(o.rho)
    for k in FIELD_KEYS:
        for i in range(nf):
            ov = getattr(o, k)[i]
            gv = g[k][i]
            # energies of a nearly empty field are compared on the total's scale
            scale = max(abs(ov), 1e-6 * rho) if k != "mean_sq" else max(abs(ov), 1e-300)
            out[f"{k}{i}"] = abs(gv - ov) / scale
    for i in range(nf):
        scale = max(abs(o.mean[i]), np.sqrt(abs(o.mean_sq[i])), 1e-300)
        out[f"mean{i}"] = abs(g["mean"][i] - o.mean[i]) / scale
    return out


def run_pair(case: Case, precision: int, steps: int, step_block: int = 32, launch=None):
    """Run the oracle and the GPU on the same seeded inputs; returns
    (gpu f, gpu fdot, gpu log dicts, oracle).  `launch`: optional
    (kernel, lanes_per_row, planes, grid) for ce_set_launch."""
    phi, phid = case.inputs()
    phi_r, phid_r = rounded(phi, precision), rounded(phid, precision)
    orc = Oracle(case.oracle_params(), phi_r, phid_r)
    orc.step(steps)
    with case.sim(precision) as s:
        if launch is not None:
            s.set_launch(*launch)
        s.set_step_block(step_block)
        s.load(phi, phid)
        s.step(steps)
        f, fd = s.read()
        log = [e.as_dict(case.nfields) for e in s.energy_log(min(steps + 1, ce.ENERGY_LOG))]
    return f, fd, log, orc
