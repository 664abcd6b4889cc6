"""The benchmark reports HBM traffic and VALU counts from the committed
rocprofv3 counter summary only while the fused kernel is built from what
the summary was taken with: its sources and device flags hash to the value
recorded there.  Host-only checks (no GPU)."""
import os
import re

import bench
from paper_2207_04658_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2207_04658_amd", "csrc")


def local_includes(path, seen):
    for name in re.findall(r'^\s*#include\s+"([^"]+)"', open(path).read(), re.M):
        full = os.path.join(os.path.dirname(path), name)
        if full not in seen:
            seen.add(full)
            if os.path.exists(full):
                local_includes(full, seen)
    return seen


def test_hash_covers_every_kernel_source():
    """Every local header the fused kernel and its run-time specialization
    include is hashed; jit_sources.inc is generated from the hashed headers
    (build.JIT_HEADERS) and the hashed device flags."""
    hashed = {os.path.normpath(os.path.join(ROOT, p)) for p in bench.KERNEL_SOURCES}
    roots = [os.path.join(CSRC, "substep.hpp"), os.path.join(CSRC, "jit.hip")]
    seen = set()
    for r in roots:
        local_includes(r, seen)
    generated = os.path.normpath(os.path.join(CSRC, "jit_sources.inc"))
    for f in {os.path.normpath(p) for p in seen} | {os.path.normpath(r) for r in roots}:
        if f == generated:
            continue
        assert f in hashed, f"{f} is compiled into the fused kernel but not hashed"
    for h in build.JIT_HEADERS:
        assert os.path.normpath(os.path.join(CSRC, h)) in hashed, h


def test_traffic_only_for_matching_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "substep_c3_counters.md")
    txt = open(path).read()
    recorded = re.search(r"kernel_sources_sha256_16:\s*([0-9a-f]+)", txt).group(1)
    hbm = float(re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt).group(1))
    valu = float(re.search(r"valu_wave_instructions_per_launch:\s*([0-9.eE+]+)", txt).group(1))
    monkeypatch.setattr(bench, "kernel_hash", lambda: recorded)
    assert bench.read_traffic("c3") == (hbm, "ok")
    assert bench.read_valu("c3") == valu
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.read_traffic("c3") == (None, "stale")
    assert bench.read_valu("c3") is None
    assert bench.read_traffic("no_such_config") == (None, None)


def test_hash_follows_sources_and_flags(monkeypatch):
    h0 = bench.kernel_hash()
    monkeypatch.setattr(build, "DEVICE_FLAGS", build.DEVICE_FLAGS + ["-DMPMQ_OTHER"])
    assert bench.kernel_hash() != h0
