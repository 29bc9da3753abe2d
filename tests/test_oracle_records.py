"""The oracle against its stored regression record (tests/golden/
oracle_records.json, written by tests/golden/make_oracle_records.py from the
oracle alone).  Not a pin: it catches unintended changes to the oracle's
arithmetic, while the closed-form and invariant pins say it is right."""
import json
import math
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_oracle_records as mk  # noqa: E402

with open(os.path.join(HERE, "golden", "oracle_records.json")) as _fh:
    STORED = json.load(_fh)


def _close(x, y, rel):
    if isinstance(x, list):
        return len(x) == len(y) and all(_close(a, b, rel) for a, b in zip(x, y))
    return math.isclose(x, y, rel_tol=rel, abs_tol=1e-14)


@pytest.mark.parametrize("name", sorted(mk.CASES))
def test_oracle_matches_record(name):
    # rounding of the generator's inverse FFT may differ between NumPy builds
    # in the last bits; 200 steps of these runs keep such differences far
    # below 1e-9
    now = mk.record(mk.CASES[name])
    assert len(now) == len(STORED[name])
    for got, want in zip(now, STORED[name]):
        assert got["step"] == want["step"]
        for key, val in want.items():
            assert _close(got[key], val, 1e-9), (name, got["step"], key, got[key], val)
