"""Streaming ceilings of the GPU's memory system, measured with the library's
probe kernel (ce_stream_probe): the best read+write copy, read-only and
write-only rates over a sweep of split, loads in flight, nontemporal hints and
grid size.  The step pass reads and writes every array once per step, so the
read+write copy rate is the rate it can at best reach; the HBM peak of the
data sheet is the other denominator.

    python -m paper_0712_0813_amd.ceiling            # compact sweep
    python -m paper_0712_0813_amd.ceiling --full     # every combination
"""
from __future__ import annotations

import argparse
import itertools
import json
import sys
from typing import Dict, List, Tuple

from . import ce

KINDS = {"copy": ce.CE_PROBE_COPY, "read": ce.CE_PROBE_READ, "write": ce.CE_PROBE_WRITE}

# (parts, unroll, nt, blocks per CU): the configurations that came out best
# in full sweeps on MI355X, plus neighbours
COMPACT = {
    "copy": [(1, 8, 3, 64), (1, 8, 3, 32), (1, 1, 2, 4), (4, 8, 3, 64), (4, 8, 3, 32)],
    "read": [(1, 4, 1, 2), (1, 8, 1, 2), (4, 1, 1, 2), (1, 4, 1, 4)],
    "write": [(1, 8, 0, 32), (1, 4, 0, 64), (4, 8, 0, 32)],
}


def full_sweep() -> Dict[str, List[Tuple[int, int, int, int]]]:
    out = {}
    for name, kind in KINDS.items():
        cfgs = []
        for parts, unroll, nt, per_cu in itertools.product((1, 4), (1, 2, 4, 8), (0, 1, 2, 3),
                                                            (2, 4, 8, 16, 32, 64)):
            if kind == ce.CE_PROBE_READ and nt & 2:
                continue
            if kind == ce.CE_PROBE_WRITE and nt & 1:
                continue
            cfgs.append((parts, unroll, nt, per_cu))
        out[name] = cfgs
    return out


def measure(torch, gib: int = 8, full: bool = False, reps: int = 5, verbose: bool = False) -> dict:
    """Best GB/s per kind (copy counts read + write bytes) over the sweep, with
    the configuration that reached it.  Uses two `gib` GiB device buffers."""
    n = gib * 1024 ** 3
    x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sweep = full_sweep() if full else COMPACT
    out = {"bytes": n, "compute_units": cus, "sweep": "full" if full else "compact"}
    for name, cfgs in sweep.items():
        kind = KINDS[name]
        best = None
        for parts, unroll, nt, per_cu in cfgs:
            ms = ce.ce_stream_probe(kind, x.data_ptr(), y.data_ptr(), n, parts=parts, unroll=unroll, nt=nt,
                                    grid=per_cu * cus, reps=reps)
            gbs = (2.0 if kind == ce.CE_PROBE_COPY else 1.0) * n / (ms / 1e3) / 1e9
            if verbose:
                print(f"{name} parts={parts} unroll={unroll} nt={nt} per_cu={per_cu}: {ms:.4f} ms "
                      f"{gbs:.1f} GB/s", file=sys.stderr, flush=True)
            if best is None or gbs > best["GBps"]:
                best = {"GBps": gbs, "ms": ms, "parts": parts, "unroll": unroll, "nt": nt, "per_cu": per_cu}
        out[name] = best
    # the copy must have moved the data
    y.zero_()
    ce.ce_stream_probe(ce.CE_PROBE_COPY, x.data_ptr(), y.data_ptr(), n, reps=1)
    torch.cuda.synchronize()
    if not torch.equal(x, y):
        raise RuntimeError("probe copy did not reproduce its source")
    del x, y
    torch.cuda.empty_cache()
    return out


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gib", type=int, default=8)
    ap.add_argument("--full", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(measure(torch, args.gib, args.full, verbose=args.verbose)), flush=True)


if __name__ == "__main__":
    main()
