"""The JSON line of bench.py on the GPU (a short run of the main line): the
fields of the benchmark line, the roofline of the timed kernel against its
own timing, and the build record of the in-tree library it loaded."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "10", "--warmup", "5",
                        "--no-cpu", "--no-extras"], capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    d = json.loads(r.stdout.strip().splitlines()[-1])
    print(json.dumps({k: d[k] for k in ("value", "ms_per_step", "roofline")}), flush=True)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "timing",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "build"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 10 and d["warmup"] == 5
    assert d["unit"] == "MLUPS" and d["higher_is_better"] is True and d["dtype"] == "f64"
    # value: lattice updates of the 256^3 box per second over the timed
    # region, the same timing as ms_per_step
    assert d["value"] > 0 and abs(d["value"] * d["ms_per_step"] * 1e3 / 256 ** 3 - 1) < 1e-3
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["kernel"] == "k_step_ab_pairs<D3Q19,f64>" and rf["bytes_per_update"] == 304
    # achieved = 304 B x 256^3 per launch over the mean launch duration
    assert abs(rf["achieved"] * rf["launch_ms_mean"] * 1e6 / (304 * 256 ** 3) - 1) < 1e-3
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert 0.3 < rf["frac"] < 1.0
    b = d["build"]
    with open(os.path.join(ROOT, b["library"]), "rb") as fh:
        assert hashlib.sha256(fh.read()).hexdigest() == b["library_sha256"]
    assert str(b["arch"]).startswith("gfx950")
