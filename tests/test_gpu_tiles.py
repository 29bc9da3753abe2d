"""The tiled 3-D pass forms its FP64 volume sums per tile and adds them in
tile order, so for one tiling (tile shape and chunk length) no result depends
on the grid or on which block worked which tile.  Lone runs whose blocks take
their tiles from the per-XCD counters (more tiles than blocks, grid a multiple
of 8), from the single counter (grid not a multiple of 8), one tile per block,
and with idle blocks, and pool members of the same tiling on two grids, all
end bitwise equal: fields, derivatives and every step's diagnostics.  The
common result matches the oracle at the parity bars.
"""
import numpy as np
import pytest

from paper_0712_0813_amd import ce
from _parity import TOL_MEAN, TOL_SITE, Case, energy_errors, site_error
from oracle import Oracle

pytestmark = pytest.mark.gpu

CASE = Case("tiles64_exp", 3, 64, 2, 10.0, 0.01, G=(0.0, 300.0, 0.0), expansion=True, seed=31)
STEPS = 30
# 64 x 16 tiles (4 sites per thread, 16 lanes per row, 256 threads) and
# 8-plane chunks: 1 x 4 x 8 = 32 tiles
SHAPE = (ce.CE_KERNEL_TILED3D, 4, 16, 256, 8)
# 8 and 16: tiles from the per-XCD counters; 12: from the single counter;
# 32: one tile per block; 40: eight blocks without a tile
LONE_GRIDS = (8, 16, 12, 32, 40)
MEMBER_GRIDS = (32, 8)


def _lone(precision, grid, phi, phid):
    with CASE.sim(precision) as s:
        s.set_launch(*SHAPE, grid)
        assert s.get_launch().as_tuple() == (*SHAPE, grid)
        s.load(phi, phid)
        s.step(STEPS)
        f, fd = s.read()
        log = [e.as_dict(CASE.nfields) for e in s.energy_log(STEPS + 1)]
    return f, fd, log


@pytest.mark.parametrize("precision", [ce.CE_FP32, ce.CE_FP64], ids=["fp32", "fp64"])
def test_tiled_result_does_not_depend_on_grid(precision):
    phi, phid = CASE.inputs()
    runs = {g: _lone(precision, g, phi, phid) for g in LONE_GRIDS}
    f0, fd0, log0 = runs[LONE_GRIDS[0]]
    for g, (f, fd, log) in runs.items():
        assert np.array_equal(f, f0) and np.array_equal(fd, fd0), f"grid {g}"
        assert log == log0, f"grid {g}"

    with ce.Pool(8 << 30) as pool:
        ids = {g: pool.admit(CASE.params(precision), phi, phid, STEPS, launch=(*SHAPE, g))
               for g in MEMBER_GRIDS}
        blocks = 0
        while pool.info().active > 0:
            pool.run_block(16)
            blocks += 1
            assert blocks < 10
        finals = {g: pool.poll(j)[1].as_dict(CASE.nfields) for g, j in ids.items()}
        fields = {g: pool.retire(j) for g, j in ids.items()}
    for g in MEMBER_GRIDS:
        pf, pfd = fields[g]
        assert np.array_equal(pf, f0) and np.array_equal(pfd, fd0), f"member grid {g}"
        assert finals[g] == log0[-1], f"member grid {g}"

    orc = Oracle(CASE.oracle_params(), phi, phid)
    orc.step(STEPS)
    for i in range(CASE.nfields):
        assert site_error(f0[i], orc.f[i]) <= TOL_SITE[precision]
        assert site_error(fd0[i], orc.pi[i]) <= TOL_SITE[precision]
    for g, o in zip(log0, orc.log):
        errs = energy_errors(g, o, CASE.nfields)
        assert max(errs.values()) <= TOL_MEAN[precision], errs
