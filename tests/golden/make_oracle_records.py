"""Writes ``oracle_records.json``: the oracle's scalar diagnostics along four
small seeded runs (1-, 2- and 3-D; rigid and self-consistent expansion; a
tachyonic double well with its vacuum energy).

The paper prints no numeric values for the evolution, so these records pin
nothing by themselves: the oracle is pinned by closed forms, invariants and
brute force in ``test_oracle_*.py``.  They are a regression record, so that
any change to the oracle's arithmetic shows up in ``test_oracle_records.py``
and has to be justified when the file is rewritten.  Only ``oracle`` is
called; inputs come from the oracle's own counter-based generator.

    python tests/golden/make_oracle_records.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle, OracleParams, grf_initial  # noqa: E402

KAPPA = 8.0 * np.pi * 0.342 ** 2
STEPS = (0, 50, 100, 200)

CASES = {
    "d1_N64_expanding": dict(
        params=OracleParams(dims=1, N=64, nfields=1, L=20.0, dt=0.01, expansion=True, kappa=KAPPA),
        seed=11, m_eff2=(1.0,), background=(1.0, 0.0, 0.0)),
    "d2_N32_two_fields_rigid": dict(
        params=OracleParams(dims=2, N=32, nfields=2, L=10.0, dt=0.01, G=(0.0, 100.0)),
        seed=12, m_eff2=(1.0, 100.0), background=(1.0, 0.0, 0.0)),
    "d3_N16_two_fields_expanding": dict(
        params=OracleParams(dims=3, N=16, nfields=2, L=10.0, dt=0.01, G=(0.0, 1000.0), expansion=True,
                            kappa=KAPPA),
        seed=13, m_eff2=(1.0, 1000.0), background=(1.0, 0.0, 0.0)),
    "d3_N16_tachyonic_vacuum": dict(
        params=OracleParams(dims=3, N=16, nfields=1, L=10.0, dt=0.01, mu2=(-1.0,), vacuum=0.25,
                            expansion=True, kappa=0.05),
        seed=14, m_eff2=(1.0,), background=(0.2, 0.0, 0.0)),
}

FIELDS = ("step", "tau", "a", "adot", "kin", "grad", "pot", "rho", "mean", "mean_sq", "resid")


def record(case: dict) -> list:
    p = case["params"]
    phi, phidot = grf_initial(case["seed"], p.dims, p.N, p.L, p.nfields, case["m_eff2"],
                              background=case["background"])
    orc = Oracle(p, phi, phidot)
    out, done = [], 0
    for k in STEPS:
        st = orc.step(k - done, record=False)
        done = k
        row = {name: getattr(st, name) for name in FIELDS}
        row["pi_sum"] = float(orc.pi.sum())
        row["pi_sq"] = float((orc.pi * orc.pi).sum())
        out.append(row)
    return out


def main():
    recs = {name: record(case) for name, case in CASES.items()}
    with open(os.path.join(HERE, "oracle_records.json"), "w") as fh:
        json.dump(recs, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
