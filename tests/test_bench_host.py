"""Host-side logic of the benchmark driver (CPU only): the hardware-counter
traffic table is used only for the kernel sources it was taken on, and a
request for more than one GPU is refused with a message."""

import json
import math
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_table_matches_current_sources():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        t = json.load(fh)
    got = bench.measured_traffic(t["dtype"])
    if t["source_sha256"] == bench.source_digest():
        assert set(got) == set(t["phases"])
        for k, v in t["phases"].items():
            assert got[k] == v["hbm_bytes_per_launch"] > 0
    else:
        assert got == {}


def test_traffic_table_ignored_for_other_sources_or_dtype(monkeypatch):
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 64)
    assert bench.measured_traffic("f32x") == {}
    monkeypatch.undo()
    assert bench.measured_traffic("no-such-dtype") == {}


def test_source_digest_is_stable():
    assert bench.source_digest() == bench.source_digest()
    assert len(bench.source_digest()) == 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_divergence_flag_uses_residual_growth():
    import numpy as np
    assert not bench.diverged(np.array([1.0, 0.5, 0.4, 0.41]))
    assert bench.diverged(np.array([1.0, 0.5, 1.2]))           # grows past ||g||
    assert bench.diverged(np.array([1.0, np.inf]))
    assert bench.diverged(np.array([1.0, np.nan, 0.1]))
    assert not bench.diverged(None)


def test_algorithmic_bytes_follow_the_per_step_convention():
    # 12 (r = g - A x) + 8 (y = A' r) + 16 (transforms read y, d, x, write x)
    assert bench.STEP_BYTES == 36
    assert bench.ALG_BYTES["row_fwd"] + bench.ALG_BYTES["col"] + bench.ALG_BYTES["row_inv"] == 16
    assert bench.FP32_VECTOR_TFLOPS == 157.3 and bench.FP64_VECTOR_TFLOPS == 78.6


def test_step_flops_follow_the_convention():
    # 4 P + F_T + 3 with F_T = 2 axes x 2 directions x 5 log2(2 (n - 1)):
    # 1,123 flops per pixel-iteration at 1024^2 with a 15 x 15 PSF
    f = bench.step_flops(1024, 1024, 225)
    assert abs(f - (900 + 20 * math.log2(2046) + 3)) < 1e-9
    assert 1122 < f < 1124
