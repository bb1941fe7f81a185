"""Host logic of bench.py that decides whether committed counter summaries
still describe the kernel being timed (no GPU needed)."""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import pytest  # noqa: E402


def test_code_only_ignores_comments_and_spacing():
    a = "int f(int x) {  // add one\n  return x + 1; /* done */\n}\n"
    b = "int f(int x) {\n\n    return x + 1;\n}  // a different comment\n"
    c = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_source_hash_is_per_precision_and_stable():
    h64, h32 = bench.kernel_source_hash("fp64"), bench.kernel_source_hash("fp32")
    assert h64 != h32
    assert h64 == bench.kernel_source_hash("fp64")
    for fam in bench.STAGE_SOURCES:
        for f in bench.STAGE_SOURCES[fam]:
            assert os.path.exists(os.path.join(ROOT, f)), f


def test_committed_traffic_matches_current_kernels():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    assert rec, "no counter records"
    stale = []
    for key, ent in rec.items():
        workload, family = key.split(":")
        assert family in bench.STAGE_SOURCES, key
        assert os.path.exists(os.path.join(ROOT, ent["summary"]))
        if ent["kernel_src"] != bench.kernel_source_hash(family):
            stale.append(key)
            continue
        assert bench.measured_traffic(workload, family, ent["options"]) == ent["bytes_per_launch"], key
        # other options (a different visiting order or tile set) are not what was measured
        other = dict(ent["options"], extra=1)
        assert bench.measured_traffic(workload, family, other) is None
        # measured traffic is at least the algorithmic bytes
        assert ent["bytes_per_launch"] >= ent["alg_bytes_per_launch"]
    if stale:
        pytest.skip(f"{stale}: kernel code changed since the counters were taken (bench reports null)")
