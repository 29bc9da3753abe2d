"""The autotuner times real launch configurations and its choices stay exact."""
import json
import os

import numpy as np
import pytest

from paper_0712_0813_amd import autotune, ce
from _parity import TOL_SITE, Case, run_pair, site_error

pytestmark = pytest.mark.gpu


def test_tune_single_and_pool(tmp_path):
    cache = str(tmp_path / "tune.json")
    e = autotune.tune(3, 64, 2, steps=3, warmup=1, cache_path=cache)
    assert e["screened"] >= 5 and 1 <= e["finalists"] <= 5 and e["ms_per_step"] > 0
    cfg = autotune.lookup(3, 64, 2, cache_path=cache)
    assert tuple(e["launch"]) == cfg
    p = autotune.tune_pool(3, 32, 1, count=4, block=3, cache_path=cache)
    assert autotune.lookup(3, 32, 1, pool=True, cache_path=cache) == tuple(p["launch"])
    data = json.load(open(cache))
    assert len(data) == 2
    # the tuned configuration still matches the oracle
    case = Case("tuned", 3, 64, 2, 2.5, 0.005, G=(0.0, 1000.0, 0.0), expansion=True, seed=4)
    f, fd, log, orc = run_pair(case, ce.CE_FP32, 100, launch=cfg)
    for i in range(2):
        assert site_error(f[i], orc.f[i]) <= TOL_SITE[ce.CE_FP32]
        assert site_error(fd[i], orc.pi[i]) <= TOL_SITE[ce.CE_FP32]
