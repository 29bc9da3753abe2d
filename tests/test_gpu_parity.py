"""GPU (HIP, through the C ABI) against the FP64 oracle on seeded inputs.

Per site after 200 steps: FP64 storage within 1e-12, FP32 storage within 1e-4
(relative, floored by the field's rms).  Diagnostics every step: 1e-11 / 1e-4.
Both sides start from the same FP64 inputs, so the representation error of
the FP32 state is part of what is measured.
"""
import numpy as np
import pytest

from paper_0712_0813_amd import ce
from paper_0712_0813_amd.workloads import DEFAULT_KAPPA, LATTICE32_STATIC
from _parity import (TOL_MEAN, TOL_SITE, Case, energy_errors, rounded, run_pair, site_error)

pytestmark = pytest.mark.gpu

W = LATTICE32_STATIC
CASES = [
    # the 32^3 static two-field workload itself
    Case("cube32_static", W.dims, W.N, W.nfields, W.L, W.dt, G=tuple(W.G), seed=W.seed),
    # 256^3-workload physics (dx = 20/256, dt = 0.005, expansion) on 32^3
    Case("cube32_expanding", 3, 32, 2, 2.5, 0.005, G=(0.0, 100.0, 0.0), expansion=True),
    # 1024^3-workload physics (dx = 40/1024, G = 1000) on 48^3: ragged block count
    Case("cube48_expanding_g1000", 3, 48, 2, 48 * 40.0 / 1024, 0.005, G=(0.0, 1000.0, 0.0),
         expansion=True, seed=1),
    # three fields, masses, 2-D
    Case("square64_3f_mass", 2, 64, 3, 10.0, 0.01, G=(0.0, 50.0, 200.0), mu2=(0.1, 0.2, 0.3),
         expansion=True, seed=5),
    Case("line256_1f_mass", 1, 256, 1, 20.0, 0.01, mu2=(0.5, 0.0, 0.0), expansion=True, seed=6),
    # smallest lattice (one quad per row) and a non-power-of-two edge
    Case("cube4_min", 3, 4, 2, 1.0, 0.01, G=(0.0, 30.0, 0.0), expansion=True, seed=7, amp=0.05),
    Case("cube12_ragged", 3, 12, 2, 3.0, 0.01, G=(0.0, 100.0, 0.0), seed=8, amp=0.01),
    Case("line4_min", 1, 4, 3, 1.0, 0.01, G=(0.0, 10.0, 20.0), seed=9, amp=0.05),
]


@pytest.mark.parametrize("precision", [ce.CE_FP64, ce.CE_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_parity_200_steps(case, precision):
    steps = 200
    f, fd, log, orc = run_pair(case, precision, steps)
    tol = TOL_SITE[precision]
    for i in range(case.nfields):
        ef = site_error(f[i], orc.f[i])
        ep = site_error(fd[i], orc.pi[i])
        assert ef <= tol, (case.name, i, "f", ef)
        assert ep <= tol, (case.name, i, "fdot", ep)
    assert len(log) == steps + 1
    tolm = TOL_MEAN[precision]
    for k, (g, o) in enumerate(zip(log, orc.log)):
        assert g["step"] == o.step == k
        errs = energy_errors(g, o, case.nfields)
        worst = max(errs, key=errs.get)
        assert errs[worst] <= tolm, (case.name, k, worst, errs[worst])
        if case.expansion:
            # r = (a'^2 - kappa rho/3)/a'^2 moves by about the relative error of rho
            assert abs(g["friedmann_residual"] - o.resid) <= tolm


TILED_CASE = Case("cube64_expanding_g1000", 3, 64, 2, 64 * 40.0 / 1024, 0.005, G=(0.0, 1000.0, 0.0),
                  expansion=True, seed=3)
T3 = ce.CE_KERNEL_TILED3D
LAUNCHES = [
    (T3, 4, 16, 256, 16, 0),   # 64x16 tile, 16 planes, resident grid
    (T3, 4, 16, 256, 64, 3),   # whole z column per tile, 3 blocks walk 4 tiles
    (T3, 4, 8, 256, 32, 0),    # 32x32 tile
    (T3, 4, 8, 256, 8, 1),     # one block walks every tile
    (T3, 2, 32, 256, 16, 0),   # two sites per thread, 64x8 tile
    (T3, 2, 32, 512, 32, 5),   # 64x16 tile, 512 threads, ragged grid
    (T3, 2, 16, 256, 64, 0),   # 32x16 tile
    (T3, 2, 16, 512, 16, 16),  # 32x32 tile, 512 threads
    (T3, 4, 16, 256, 24, 0),   # z column cut into chunks of 21, 21 and 22 planes
    (T3, 2, 32, 256, 27, 5),   # uneven chunks, ragged grid
    (ce.CE_KERNEL_DIRECT, 0, 0, 0, 0, 7),  # direct kernel, ragged grid
]


@pytest.mark.parametrize("precision", [ce.CE_FP64, ce.CE_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("launch", LAUNCHES, ids=lambda l: "k%d_v%d_l%d_b%d_z%d_g%d" % l)
def test_launch_configs_parity(launch, precision):
    case = TILED_CASE
    steps = 200
    f, fd, log, orc = run_pair(case, precision, steps, launch=launch)
    tol = TOL_SITE[precision]
    for i in range(case.nfields):
        assert site_error(f[i], orc.f[i]) <= tol, (i, "f", site_error(f[i], orc.f[i]))
        assert site_error(fd[i], orc.pi[i]) <= tol, (i, "fdot", site_error(fd[i], orc.pi[i]))
    for k, (g, o) in enumerate(zip(log, orc.log)):
        errs = energy_errors(g, o, case.nfields)
        worst = max(errs, key=errs.get)
        assert errs[worst] <= TOL_MEAN[precision], (k, worst, errs[worst])


S2 = ce.CE_KERNEL_STREAM2D
SQUARE_CASE = Case("square256_expanding_g100", 2, 256, 2, 40.0, 0.01, G=(0.0, 100.0, 0.0),
                   expansion=True, seed=12)
STREAM2D_LAUNCHES = [
    (S2, 4, 64, 256, 64, 0),   # four units, one block
    (S2, 4, 64, 256, 8, 0),    # 32 units, resident grid
    (S2, 4, 64, 256, 16, 3),   # ragged grid: blocks walk several groups
    (S2, 4, 64, 256, 1, 8),    # one row per unit, XCD-contiguous group order
    (S2, 4, 64, 256, 256, 1),  # one unit holds the lattice; three waves idle
    (ce.CE_KERNEL_DIRECT, 0, 0, 0, 0, 0),
]


@pytest.mark.parametrize("precision", [ce.CE_FP64, ce.CE_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("launch", STREAM2D_LAUNCHES, ids=lambda l: "k%d_z%d_g%d" % (l[0], l[4], l[5]))
def test_stream2d_launches_parity(launch, precision):
    case = SQUARE_CASE
    steps = 200
    f, fd, log, orc = run_pair(case, precision, steps, launch=launch)
    tol = TOL_SITE[precision]
    for i in range(case.nfields):
        assert site_error(f[i], orc.f[i]) <= tol, (i, "f", site_error(f[i], orc.f[i]))
        assert site_error(fd[i], orc.pi[i]) <= tol, (i, "fdot", site_error(fd[i], orc.pi[i]))
    for k, (g, o) in enumerate(zip(log, orc.log)):
        errs = energy_errors(g, o, case.nfields)
        worst = max(errs, key=errs.get)
        assert errs[worst] <= TOL_MEAN[precision], (k, worst, errs[worst])
        assert abs(g["friedmann_residual"] - o.resid) <= TOL_MEAN[precision]


def test_stream2d_segments_and_three_fields():
    # two 256-site segments per row: the edge lanes read across segments
    case = Case("square512_3f_mass", 2, 512, 3, 60.0, 0.01, G=(0.0, 30.0, 2000.0),
                mu2=(0.2, 0.0, 0.5), expansion=True, seed=13)
    for precision, launch in ((ce.CE_FP64, (S2, 4, 64, 256, 32, 0)), (ce.CE_FP32, (S2, 4, 64, 256, 8, 5))):
        f, fd, log, orc = run_pair(case, precision, 120, launch=launch)
        tol = TOL_SITE[precision]
        for i in range(3):
            assert site_error(f[i], orc.f[i]) <= tol, (precision, i, "f")
            assert site_error(fd[i], orc.pi[i]) <= tol, (precision, i, "fdot")
        for k, (g, o) in enumerate(zip(log, orc.log)):
            errs = energy_errors(g, o, 3)
            worst = max(errs, key=errs.get)
            assert errs[worst] <= TOL_MEAN[precision], (precision, k, worst, errs[worst])


def test_stream2d_matches_direct_kernel():
    # the per-site arithmetic is the direct kernel's; only the order of the
    # volume sums differs, so the two agree far inside the oracle tolerance
    case = SQUARE_CASE
    phi, phid = case.inputs()
    outs = []
    for launch in ((S2, 4, 64, 256, 16, 0), (ce.CE_KERNEL_DIRECT, 0, 0, 0, 0, 0)):
        with case.sim(ce.CE_FP32) as s:
            s.set_launch(*launch)
            s.load(phi, phid)
            s.step(20)
            outs.append((s.read(), s.energies().as_dict(2)))
    (f0, fd0), e0 = outs[0]
    (f1, fd1), e1 = outs[1]
    for i in range(2):
        assert site_error(f0[i], f1[i]) <= 1e-6, (i, site_error(f0[i], f1[i]))
        assert site_error(fd0[i], fd1[i]) <= 1e-6, (i, site_error(fd0[i], fd1[i]))
    assert abs(e0["rho"] - e1["rho"]) <= 1e-9 * abs(e1["rho"])


def test_tiled_three_fields_fp64():
    case = Case("cube64_3f_mass", 3, 64, 3, 6.0, 0.01, G=(0.0, 30.0, 300.0), mu2=(0.2, 0.0, 0.5),
                expansion=True, seed=11)
    f, fd, log, orc = run_pair(case, ce.CE_FP64, 200, launch=(T3, 4, 16, 256, 32, 0))
    for i in range(3):
        assert site_error(f[i], orc.f[i]) <= 1e-12
        assert site_error(fd[i], orc.pi[i]) <= 1e-12
    f, fd, log, orc = run_pair(case, ce.CE_FP32, 200, launch=(T3, 2, 16, 512, 16, 0))
    for i in range(3):
        assert site_error(f[i], orc.f[i]) <= 1e-4
        assert site_error(fd[i], orc.pi[i]) <= 1e-4


def test_default_launch_choice():
    big = Case("cube256", 3, 256, 2, 10.0, 0.01, G=(0.0, 100.0, 0.0))
    with big.sim(ce.CE_FP32) as s:
        cfg = s.get_launch()
        assert cfg.kernel == ce.CE_KERNEL_TILED3D and cfg.grid >= 256
    with SQUARE_CASE.sim(ce.CE_FP32) as s:
        cfg = s.get_launch()
        assert cfg.kernel == S2 and cfg.as_tuple()[1:4] == (4, 64, 256) and 256 % cfg.planes == 0
        with pytest.raises(ce.CeError):
            s.set_launch(S2, 4, 64, 256, 3, 0)  # rows must divide N
    with CASES[3].sim(ce.CE_FP32) as s:  # 2-D, N = 64: no whole 256-site segment
        assert s.get_launch().kernel == ce.CE_KERNEL_DIRECT
        with pytest.raises(ce.CeError):
            s.set_launch(S2, 4, 64, 256, 8, 0)
    with CASES[0].sim(ce.CE_FP32) as s:
        assert s.get_launch().kernel == ce.CE_KERNEL_DIRECT
        with pytest.raises(ce.CeError):
            s.set_launch(S2, 4, 64, 256, 8, 0)  # 3-D
        with pytest.raises(ce.CeError):
            s.set_launch(T3, 2, 32, 256, 33, 0)  # more planes than N
        with pytest.raises(ce.CeError):
            s.set_launch(T3, 4, 32, 256, 16, 0)  # shape not built
        assert s.get_launch().kernel == ce.CE_KERNEL_DIRECT


def test_step_blocks_match_plain_launches_bitwise():
    case = CASES[1]
    phi, phid = case.inputs()
    outs = []
    for block in (0, 7, 32):
        with case.sim(ce.CE_FP32) as s:
            s.set_step_block(block)
            s.load(phi, phid)
            s.step(3)
            s.step(70)
            outs.append((s.read(), s.energies().as_dict(2)))
    for (f, fd), e in outs[1:]:
        assert np.array_equal(f, outs[0][0][0]) and np.array_equal(fd, outs[0][0][1])
        assert e == outs[0][1]


def test_run_twice_bitwise():
    case = CASES[2]
    phi, phid = case.inputs()
    res = []
    for _ in range(2):
        with case.sim(ce.CE_FP32) as s:
            s.load(phi, phid)
            s.step(50)
            res.append((s.read(), [e.as_dict(2) for e in s.energy_log(51)]))
    assert np.array_equal(res[0][0][0], res[1][0][0])
    assert np.array_equal(res[0][0][1], res[1][0][1])
    assert res[0][1] == res[1][1]


@pytest.mark.parametrize("precision,tol", [(ce.CE_FP64, 1e-13), (ce.CE_FP32, 1e-5)],
                         ids=["fp64", "fp32"])
def test_translation_invariance(precision, tol):
    """Shifted inputs give shifted outputs.  Exact in real arithmetic; the
    FP64 homogeneous references come from volume sums whose order follows the
    site numbering, so agreement is to rounding."""
    case = CASES[1]
    phi, phid = case.inputs()
    shift = (0, 5, 11, 3)
    outs = []
    for sh in ((0, 0, 0, 0), shift):
        with case.sim(precision) as s:
            s.load(np.roll(phi, sh, axis=(0, 1, 2, 3)), np.roll(phid, sh, axis=(0, 1, 2, 3)))
            s.step(40)
            outs.append(s.read())
    for k in range(2):
        a = np.roll(outs[0][k], shift, axis=(0, 1, 2, 3))
        b = outs[1][k]
        for i in range(case.nfields):
            assert site_error(b[i], a[i]) <= tol, (k, i, site_error(b[i], a[i]))


def test_chi_sign_symmetry_bitwise():
    case = CASES[1]
    phi, phid = case.inputs()
    s_ = np.array([1.0, -1.0])[:, None, None, None]
    outs = []
    for sg in (np.ones_like(s_), s_):
        with case.sim(ce.CE_FP32) as s:
            s.load(phi * sg, phid * sg)
            s.step(30)
            outs.append(s.read())
    assert np.array_equal(outs[0][0] * s_, outs[1][0])
    assert np.array_equal(outs[0][1] * s_, outs[1][1])


def test_read_sites_matches_read_fields():
    case = CASES[2]
    phi, phid = case.inputs()
    with case.sim(ce.CE_FP32) as s:
        s.load(phi, phid)
        s.step(9)
        f, fd = s.read()
        sites = np.random.default_rng(0).integers(0, case.N ** 3, 1000)
        for i in range(2):
            a, b = s.read_sites(i, sites)
            assert np.array_equal(a, f[i].ravel()[sites]) and np.array_equal(b, fd[i].ravel()[sites])


def test_state_errors():
    case = CASES[0]
    with case.sim(ce.CE_FP32) as s:
        with pytest.raises(ce.CeError) as ei:
            s.step(1)
        assert ei.value.status == ce.CE_ESTATE
        phi, phid = case.inputs()
        s.load(phi[:1], phid[:1], first=0)  # one of two fields: still not started
        with pytest.raises(ce.CeError):
            s.step(1)
        s.load(phi[1:], phid[1:], first=1)
        s.step(2)
        assert s.step_count == 2
        assert s.energies().step == 2


def test_nonfinite_is_reported():
    case = CASES[0]
    phi, phid = case.inputs()
    phid[1, 3, 4, 5] = 1e30  # finite input, overflows FP32 at once
    with case.sim(ce.CE_FP32) as s:
        s.load(phi, phid)
        s.step(5)
        with pytest.raises(ce.CeError) as ei:
            s.energies()
        assert ei.value.status == ce.CE_ENONFINITE
        e = s.energies(allow_nonfinite=True)
        assert e.step == 5


def test_nonfinite_initial_data_rejected():
    # 64^3: the homogeneous reference samples every 4th site; the NaN sits
    # between samples and must still be caught
    case = TILED_CASE
    for field, kind in ((0, "phi"), (1, "phi"), (1, "phidot")):
        phi, phid = case.inputs()
        (phi if kind == "phi" else phid)[field, 3, 17, 29] = np.nan
        with case.sim(ce.CE_FP32) as s:
            with pytest.raises(ce.CeError) as ei:
                s.load(phi, phid)
            assert ei.value.status == ce.CE_EINVAL


def test_unstable_initial_data_rejected():
    case = Case("stiff", 3, 16, 2, 10.0, 0.01, G=(0.0, 1e6, 0.0))
    phi, phid = case.inputs()
    with case.sim(ce.CE_FP32) as s:
        with pytest.raises(ce.CeError) as ei:
            s.load(phi, phid)
        assert ei.value.status == ce.CE_EINVAL and "unstable" in str(ei.value)


def test_stream_copy_measurement_kernel_copies():
    import torch
    n = 64 * 2 ** 20
    x = torch.randint(0, 2 ** 31 - 1, (n // 4,), dtype=torch.int32, device="cuda")
    for streams in (1, 2, 4):
        y = torch.zeros_like(x)
        ms = ce.ce_stream_copy(x.data_ptr(), y.data_ptr(), n, streams=streams, grid=0, reps=2)
        assert ms > 0
        assert torch.equal(x, y), streams
    with pytest.raises(ce.CeError):
        ce.ce_stream_copy(x.data_ptr(), y.data_ptr(), n, streams=3)
