"""Host side of the autotuner: the candidate launches it times are all
well-formed for the lattice, include the library's defaults, and use only
tile shapes the library builds."""
import json
import os
import re

import pytest

from paper_0712_0813_amd import autotune, ce

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_shapes_match_header():
    text = open(os.path.join(ROOT, "include", "ce.h")).read()
    block = text[text.index("Tiled shapes built"):]
    block = block[:block.index("*/")]
    shapes = {tuple(int(x) for x in m) for m in re.findall(r"\((\d+),(\d+),(\d+)\)", block)}
    assert shapes == set(ce.TILED_SHAPES)


@pytest.mark.parametrize("dims,N", [(3, 32), (3, 64), (3, 256), (3, 1024), (2, 256), (2, 2048), (1, 4096)])
def test_candidates_well_formed(dims, N):
    cands = autotune.candidates(dims, N)
    assert len(cands) == len(set(cands))
    kinds = {c[0] for c in cands}
    assert ce.CE_KERNEL_DIRECT in kinds
    assert (ce.CE_KERNEL_TILED3D in kinds) == (dims == 3)
    assert (ce.CE_KERNEL_STREAM2D in kinds) == (dims == 2)
    for kind, v, lpr, block, planes, grid in cands:
        assert grid >= 0
        if kind == ce.CE_KERNEL_TILED3D:
            assert (v, lpr, block) in ce.TILED_SHAPES
            assert N % (v * lpr) == 0 and N % (block // lpr) == 0 and 2 <= planes <= N
            # ragged chunk splits run on the evened resident grid only
            assert N % planes == 0 or grid == 0
        elif kind == ce.CE_KERNEL_STREAM2D:
            assert N % 256 == 0 and N % planes == 0


def test_headline_default_is_a_candidate():
    # the 1024^3 default launch: 256 x 4 tiles in three chunks of 342, 342 and
    # 340 planes on the evened resident grid
    assert (ce.CE_KERNEL_TILED3D, 4, 64, 256, 342, 0) in autotune.candidates(3, 1024)


@pytest.mark.parametrize("N", [32, 64, 100, 256, 1024])
def test_chunk_lengths(N):
    zs = autotune.chunk_lengths(N)
    assert zs == sorted(set(zs)) and all(2 <= z <= N for z in zs)
    counts = {-(-N // z) for z in zs}
    # every split into 1..16 chunks appears once, at its shortest length
    for nz in range(1, min(N // 2, 16) + 1):
        z = -(-N // nz)
        if -(-N // z) == nz:
            assert z in zs
    assert len(counts) <= len(zs)
    if N == 1024:
        assert {1024, 512, 342, 256, 205, 128, 64, 2} <= set(zs)


@pytest.mark.parametrize("dims,N", [(3, 32), (3, 64), (3, 128), (3, 256), (2, 256), (2, 2048)])
def test_member_candidates_one_tile_per_block(dims, N):
    for kind, v, lpr, block, planes, grid in autotune.member_candidates(dims, N):
        if kind == ce.CE_KERNEL_TILED3D:
            tiles = (N // (v * lpr)) * (N // (block // lpr)) * (N // planes)
            assert grid == tiles <= 4096
        elif kind == ce.CE_KERNEL_STREAM2D:
            units = (N // 256) * (N // planes)
            assert grid == -(-units // 4) <= 4096
        else:
            assert 1 <= grid <= 2048


def test_cache_keys_and_lookup(tmp_path):
    key = autotune.class_key("gfx950", 3, 64, 2, ce.CE_FP64)
    assert key == "gfx950/d3/N64/nf2/fp64"
    path = tmp_path / "cache.json"
    h = autotune.source_hash()
    path.write_text(json.dumps({"pool/gfx950/d3/N64/nf2/fp32": {"launch": [1, 4, 16, 256, 64, 4], "source_hash": h},
                                "gfx950/d3/N64/nf2/fp32": {"launch": [1, 4, 16, 256, 64, 0], "source_hash": "0" * 16},
                                "gfx950/d3/N32/nf2/fp32": {"launch": [1, 4, 16, 256, 32, 0]}}))
    assert autotune.lookup(3, 64, 2, arch="gfx950", cache_path=str(path), pool=True) == (1, 4, 16, 256, 64, 4)
    # entries measured on other sources, or with no hash, are not used
    assert autotune.lookup(3, 64, 2, arch="gfx950", cache_path=str(path)) is None
    assert autotune.lookup(3, 32, 2, arch="gfx950", cache_path=str(path)) is None
    assert autotune.lookup(3, 64, 2, arch="gfx950", cache_path=str(tmp_path / "none.json"), pool=True) is None


def test_source_hash_follows_sources(tmp_path, monkeypatch):
    h = autotune.source_hash()
    assert len(h) == 16 and h == autotune.source_hash()
    # a copy of the package with one kernel byte changed hashes differently
    import shutil
    pkg = tmp_path / "pkg"
    shutil.copytree(os.path.join(ROOT, "paper_0712_0813_amd", "csrc"), pkg / "csrc")
    shutil.copy(os.path.join(ROOT, "paper_0712_0813_amd", "build.py"), pkg / "build.py")
    (tmp_path / "include").mkdir()
    shutil.copy(os.path.join(ROOT, "include", "ce.h"), tmp_path / "include" / "ce.h")
    monkeypatch.setattr(autotune, "_PKG", str(pkg))
    monkeypatch.setattr(autotune, "_ROOT", str(tmp_path))
    assert autotune.source_hash() == h
    f = pkg / "csrc" / "ce_step3d.hip"
    f.write_bytes(f.read_bytes() + b"\n")
    assert autotune.source_hash() != h


def test_arch_from_driver_topology(tmp_path, monkeypatch):
    """The cache key's architecture comes from the driver's node properties
    (no GPU runtime involved): the first node with a nonzero gfx target."""
    for n, v in (("0", 0), ("1", 90500), ("2", 90402)):
        d = tmp_path / n
        d.mkdir()
        (d / "properties").write_text(f"cpu_cores_count 16\ngfx_target_version {v}\nsimd_count 1024\n")
    monkeypatch.setattr(autotune, "KFD_NODES", str(tmp_path))
    assert autotune._kfd_arch() == "gfx950"
    (tmp_path / "1" / "properties").write_text("gfx_target_version 90010\n")
    assert autotune._kfd_arch() == "gfx90a"
    monkeypatch.setattr(autotune, "KFD_NODES", str(tmp_path / "missing"))
    assert autotune._kfd_arch() is None
