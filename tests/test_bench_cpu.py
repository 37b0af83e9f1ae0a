"""Host-side parts of bench.py: the oracle's CPU baseline (timed in net and
decode parts, on all threads and on one) and the one-GPU guard."""
import os
import subprocess
import sys

import numpy as np

import bench
import oracle
from paper_2202_05977_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_baseline_is_the_oracle_denoise(oracle_lib):
    cfg = synth.HD
    blob = synth.make_weights(cfg, 0)
    H, W = 48, 80
    fr = synth.make_frame(1, H, W)
    cpu, y = bench.cpu_baseline(fr, blob, cfg, H, W)
    # the two timed parts compose to exactly the oracle's whole-frame path
    assert np.array_equal(y, oracle.denoise(fr, blob, cfg))
    assert cpu["kind"] == "oracle" and cpu["unit"] == "frames/s"
    assert cpu["value"] == 1.0 / (cpu["net_s"] + cpu["decode_s"])
    assert cpu["cores"] >= 1 and cpu["one_thread"]["net_s"] > 0 and cpu["one_thread"]["decode_s"] > 0
    # the one-thread net sample is a crop the net accepts (sides multiples of 8)
    assert "x" in cpu["one_thread"]["sample"]
    assert cpu["cpu_model"]


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stdout + p.stderr
