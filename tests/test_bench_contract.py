"""bench.py's contract on the CPU: the multi-GPU request exits with a message before any device
call, the roofline counts the method's algorithmic bytes (96 B per particle for the fused
gather-kick-drift, 24 B for the deposit; the sort index reported apart), and the committed
counter summaries parse against the kernels' source text."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_are_the_methods_minimum():
    # fused gather-kick-drift: six float64 coordinates read and written; deposit: x, y, z read
    assert bench.ALGO_BYTES == {"gkd": 6 * 8 * 2, "deposit": 3 * 8}
    # the permutation's 4-byte source index is overhead, not algorithmic
    assert bench.OVERHEAD_BYTES == {"gkd": 4, "deposit": 4}


@pytest.mark.parametrize("kernel", ["gkd", "deposit"])
def test_kernel_source_text_is_found(kernel):
    rel, func = bench.KERNEL_SOURCES[kernel]
    text = bench.function_text(os.path.join(ROOT, rel), func)
    assert ("void %s(" % func) in text and text.rstrip().endswith("}")
    assert len(bench._source_hash(kernel)) == 16


@pytest.mark.parametrize("kernel", ["gkd", "deposit"])
def test_traffic_summary_parses(kernel):
    path = os.path.join(ROOT, "profiles", "traffic_%s_gausshalo-1e8-128c-tsc.txt" % kernel)
    rec = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    assert len(rec["source_sha256_16"]) == 16
    b = float(rec["bytes_per_launch"])
    # counter traffic can exceed the algorithmic bytes (over-fetch) but not fall below them
    assert b >= bench.ALGO_BYTES[kernel] * 1e8
    # _traffic reports the figure only while it was taken on the current kernel source
    t = bench._traffic(kernel, "gausshalo-1e8-128c-tsc")
    assert t is None or t == b
