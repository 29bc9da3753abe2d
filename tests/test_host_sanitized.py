"""The C-ABI library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.  The library is rebuilt with the
sanitizers on its host side only (device code as usual), and every call that
needs no GPU is driven through it in a child process: parameter validation,
including sizes whose N^dims overflows 64 bits, and the grid-image header
parser fed thousands of corrupted headers.  Any sanitizer report fails."""
import glob
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0712_0813_amd", "csrc")

# host-side sanitizers only: each -fsanitize= applies to the host pass
FLAGS = ("--offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -ffp-contract=off "
         "-Xclang -target-feature -Xclang -packed-fp32-ops "
         "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
         "-Xarch_host -fno-sanitize-recover=undefined").split()
LINK = "--offload-arch=gfx950 -shared -fPIC -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    import numpy as np
    from paper_0712_0813_amd import ce
    ce.LIB_PATH = {lib!r}
    from test_image_cpu import header
    # validation: accepted and rejected parameter sets, no device work
    for dims, N in [(3, 16), (3, 1024), (2, 2 ** 20), (1, 4096)]:
        assert ce.ce_required_bytes(ce.make_params(dims, N, 2, 1e9, 0.01)) > 0
    for dims, N in [(3, 33744500), (3, 2 ** 22), (2, 2 ** 20 + 4), (3, 30), (4, 16)]:
        try:
            ce.ce_required_bytes(ce.make_params(dims, N, 1, 1e9, 0.01))
            raise SystemExit("accepted %d %d" % (dims, N))
        except ce.CeError:
            pass
    # image headers: random corruptions and truncations, and size fields near 2^64
    good = header()
    rng = np.random.default_rng(0)
    for t in range(5000):
        buf = good.copy()
        for _ in range(int(rng.integers(1, 6))):
            buf[int(rng.integers(0, 256))] = rng.integers(0, 256)
        n = int(rng.integers(0, buf.size + 1)) if rng.random() < 0.2 else buf.size
        try:
            ce.ce_image_params(buf[:n].copy())
        except ce.CeError:
            pass
    off = {{n: getattr(ce.ce_image_header, n).offset for n, _ in ce.ce_image_header._fields_}}
    for field in ("state_bytes", "ring_bytes", "field_bytes", "total_bytes"):
        for v in (2 ** 63, 2 ** 64 - 1, 2 ** 40):
            buf = good.copy()
            buf[off[field]:off[field] + 8] = np.frombuffer(np.uint64(v).tobytes(), np.uint8)
            try:
                ce.ce_image_params(buf)
                raise SystemExit("accepted %s=%d" % (field, v))
            except ce.CeError:
                pass
    lib = ce.load_library()
    assert lib.ce_step(None, 1) == ce.CE_EINVAL
    lib.ce_destroy(None)
    print("sanitized host checks done")
""")


def test_host_library_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    runtime = _asan_runtime()
    if not os.path.exists(hipcc) or runtime is None:
        pytest.skip("hipcc or the clang sanitizer runtime is not available")
    from paper_0712_0813_amd import build as libbuild
    objs = []
    for src, extra, name in libbuild.compile_units():
        obj = str(tmp_path / name)
        r = subprocess.run([hipcc, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o",
                            obj], capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        objs.append(obj)
    lib = str(tmp_path / "libce_sanitized.so")
    r = subprocess.run([hipcc, *LINK, "-o", lib, *objs], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    child = tmp_path / "child.py"
    child.write_text(CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib))
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, str(child)], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "sanitized host checks done" in r.stdout
