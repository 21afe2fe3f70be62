"""Host-side pieces of bench.py: the single-GPU guard, the issued-MFMA
count, and the reading of committed rocprofv3 summaries (a figure is used
only while the kernel sources still hash to the value recorded with it).
Nothing here touches a device."""
import importlib.util
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_issued_mfma_flops(bench):
    # N = 64, L = 16, split-BF16: one diagonal tile, three of its four 32x32
    # blocks live (the block below the diagonal idles), 9 correlations of
    # 32 x 32 pairs over K = 16, three products, FMA = 2
    assert bench.issued_mfma_flops("bf16", 64, 16) == 3 * 32 * 32 * 9 * 16 * 2.0 * 3
    # K padded to the K-block (8 for FP32), the x4 mode's fourth product
    assert bench.issued_mfma_flops("fp32", 64, 9) == 3 * 32 * 32 * 9 * 16 * 2.0
    assert bench.issued_mfma_flops("bf16x4", 64, 16) == 3 * 32 * 32 * 9 * 16 * 2.0 * 4


def test_profile_values_follow_the_source_hash(bench, tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: "00112233aabbccdd")
    (prof / "tile_bf16_w_kernel_trace.md").write_text(
        "text\navg-ms-per-launch: 2.5\nsource-sha256: 00112233aabbccdd\n")
    (prof / "tile_bf16_w_hbm_traffic.md").write_text(
        "traffic-bytes-per-launch: 123456\nsource-sha256: ffffffffffffffff\n")
    assert bench.profile_value("bf16", "w", "kernel_trace", "avg-ms-per-launch") == 2.5
    assert bench.traffic_from_profiles("bf16", "w") is None          # stale hash
    assert bench.profile_value("bf16", "w", "counters", "mfma-busy-frac") is None


def test_committed_profiles_carry_the_fields_the_bench_reads():
    for kind, keys in (("kernel_trace", ["avg-ms-per-launch"]),
                       ("hbm_traffic", ["traffic-bytes-per-launch"]),
                       ("counters", ["mfma-busy-frac", "valu-busy-frac", "mfma-valu-coexec-frac",
                                     "valu-insts-per-pair", "fp64-insts-per-pair"])):
        txt = open(os.path.join(ROOT, "profiles", f"tile_bf16_n20000_l150_{kind}.md")).read()
        assert re.search(r"source-sha256:\s*[0-9a-f]{16}", txt), kind
        assert "rocprofv3" in txt, kind
        for k in keys:
            assert re.search(re.escape(k) + r":\s*[0-9.eE+-]+", txt), (kind, k)
