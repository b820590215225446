"""Host-side logic of bench.py (no GPU): the one-GPU guard, the oracle baseline leg and the
traffic record lookup."""
import os
import subprocess
import sys

import numpy as np

import bench
import oracle
from paper_1504_05046_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_fields_and_zero_error_on_the_oracle_result():
    p = gen.random_problem(31, 12, 12, 12, 32, 160, 0.4, 0.4)
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    cbits = oracle.shape_product(p.M, p.K, p.N, p.a_bits(), p.b_bits())
    off, total = oracle.block_offsets(p.rows, p.cols, cbits)
    assert total == ref.size
    cb, err = bench.cpu_baseline(p, ref, off, 0.5)
    assert err == 0.0
    assert cb["kind"] == "oracle" and cb["unit"] == "TFLOP/s" and cb["value"] > 0
    assert cb["cores"] == oracle.threads() >= 1
    assert isinstance(cb["cpu_model"], str) and cb["cpu_model"]
    assert cb["single_thread"]["value"] > 0
    u = cb["uniform_1024_full_product_ms"]
    assert u["single_thread"] > 0 and u["all_threads"] > 0
    assert oracle.threads() == cb["cores"]          # the thread count was restored


def test_recorded_traffic_is_positive_or_absent():
    t = bench.recorded_traffic()
    assert t is None or t > 0
