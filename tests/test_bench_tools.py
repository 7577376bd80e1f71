"""The benchmark's own contract and tooling, on the CPU: the one-GPU guard, the kernel-code
hash that keys the committed counter summaries, and the staleness rule for those summaries."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert out.stdout == ""                      # no JSON line
    assert "one GPU" in out.stderr


def test_kernel_hash_ignores_comments_only(tmp_path):
    a = tmp_path / "a.hip"
    a.write_text("// header\n__global__ void k(int* p) {\n  p[0] = 1;  // store\n\n}\n")
    b = tmp_path / "b.hip"
    b.write_text("// another header\n\n__global__ void k(int* p) {   \n  p[0] = 1;\n}\n// trailing\n")
    c = tmp_path / "c.hip"
    c.write_text("__global__ void k(int* p) {\n  p[0] = 2;\n}\n")
    assert bench.kernel_source_hash(str(a)) == bench.kernel_source_hash(str(b))
    assert bench.kernel_source_hash(str(a)) != bench.kernel_source_hash(str(c))


def test_traffic_summary_is_used_only_for_the_kernels_it_measured(tmp_path):
    # a summary in the committed format: RAW lines in KiB per launch, the copy-calibrated
    # SCALE factors and the SOURCE hash of the kernels the counters were taken on
    def summary(source):
        return ("SCALE read 2.0 write 1.0\n"
                f"SOURCE {source}\n"
                "RAW hzd::k_x fetch_KiB 100 write_KiB 10\n")
    good = tmp_path / "good.txt"
    good.write_text(summary(bench.kernel_source_hash()))
    assert bench.measured_traffic("hzd::k_x", str(good)) == round((100 * 2.0 + 10 * 1.0) * 1024)
    assert bench.measured_traffic("hzd::k_y", str(good)) is None          # not measured
    stale = tmp_path / "stale.txt"
    stale.write_text(summary("0123456789abcdef"))
    assert bench.measured_traffic("hzd::k_x", str(stale)) is None         # kernels changed since
    assert bench.measured_traffic("hzd::k_x", str(tmp_path / "missing.txt")) is None


def test_committed_summaries_name_their_kernels():
    # every summary under profiles/ records the kernel-code hash it was taken on; while it
    # matches the kernels as they are, bench.py uses the traffic figures, otherwise it reports
    # null (a kernel change without new profiles is reported here as a skip, not hidden)
    h = bench.kernel_source_hash()
    stale = []
    for name in ("traffic_1080p_offline.txt", "traffic_resize_1080p_to_640x480_x8.txt",
                 "kernels_1080p_offline.txt", "sq_counters_1080p_offline.txt",
                 "kernels_1080p_offline_x8.txt", "sq_counters_1080p_offline_x8.txt"):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "kernel code sha256[:16]" in text or "SOURCE " in text, name
        if h not in text:
            stale.append(name)
    if stale:
        pytest.skip(f"profiles taken on other kernel code: {stale}")
