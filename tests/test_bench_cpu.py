"""Host-side logic of bench.py (no GPU): the one-GPU rule, the name of the
timed kernel, and the use of the committed HBM counter figures."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_timed_kernel_name():
    assert bench.step_kernel_name(256, "f64", "ab") == "k_step_ab_pairs<D3Q19,f64>"
    assert bench.step_kernel_name(256, "f64", "aa") == "k_step_aa_pairs<D3Q19,f64>"
    assert bench.step_kernel_name(256, "f16", "ab") == "k_step_ab<D3Q19,f16>"
    assert bench.step_kernel_name(255, "f64", "ab") == "k_step_ab<D3Q19,f64>"  # odd nx
    assert bench.step_kernel_name(64, "f64", "ab") == "k_step_ab<D3Q19,f64>"   # < 2^20 nodes
    # FP32 and e4m11 two-lattice steps on rows of a power-of-two length
    assert bench.step_kernel_name(512, "e4m11", "ab") == "k_step_ab_rows<D3Q19,e4m11>"
    assert bench.step_kernel_name(128, "f32", "ab") == "k_step_ab_rows<D3Q19,f32>"
    assert bench.step_kernel_name(96, "f32", "ab") == "k_step_ab<D3Q19,f32>"
    assert bench.step_kernel_name(256, "e4m11", "aa") == "k_step_aa<D3Q19,e4m11>"


def test_counter_figures_follow_the_kernel_sources():
    """roofline.traffic comes from the committed counters only while the step
    kernels' sources hash to the value recorded with them; otherwise null."""
    path = os.path.join(ROOT, "profiles", "k_step_ab_pairs_d3q19_f64_256cube.counters.json")
    with open(path) as fh:
        d = json.load(fh)
    got = bench.measured_traffic("f64", "ab", 256)
    if d["sources_sha256"] == bench.kernel_sources_sha256():
        assert got == d["traffic_bytes_per_launch"]
        # the figures themselves: traffic within 0.1 % of 304 B per node
        assert abs(got / (304 * 256 ** 3) - 1) < 1e-3
    else:
        assert got is None
    assert bench.measured_traffic("f64", "ab", 128) is None  # no figures for that box
