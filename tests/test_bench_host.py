"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte and flop counts behind the roofline record (checked against independent
counts), and that solutions are copied for the oracle check only when it runs.
"""
import os
import subprocess
import sys

import bench
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_dst_bytes_per_launch():
    """One DST pass reads and writes the spectrum of real time data once: n/2 - 1
    complex blocks and the two real ones, i.e. n m values, FP64."""
    w = W.WORKLOADS["heat2d_255x256"]
    assert bench.class_bytes(w, "fp64")["dst"] == 2 * 256 * 255 * 255 * 8 == 266342400


def test_dst_launch_mix_and_flops():
    """255^2 x 256 FP64: x forward, fused last axis (forward, divide, inverse),
    x inverse = 3 launches for 4 products.  The two-level fold runs a quarter
    of the dense DST-I multiply-adds (FP64 and FP32 alike at odd m and a padded
    length that is a multiple of 128; P = 512 has no fused kernel)."""
    w = W.WORKLOADS["heat2d_255x256"]
    assert bench.dst_path(w, "fp64") == "fold2"
    assert bench.dst_launch_mix(w, "fp64") == (3, 4)
    md = w.m1
    dense_flops = 2.0 * md * md * w.n * (w.m // md)
    assert abs(bench.dst_product_flops(w, "fp64") / dense_flops - 0.25) < 0.005
    w32 = W.WORKLOADS["heat2d_511x512"]
    assert bench.dst_path(w32, "fp32") == "fold2"
    assert bench.dst_launch_mix(w32, "fp32") == (4, 4)
    assert bench.dst_launch_mix(w, "fp32") == (3, 4)
    dense32 = 2.0 * w32.m1 ** 2 * w32.n * (w32.m // w32.m1)
    assert abs(bench.dst_product_flops(w32, "fp32") / dense32 - 0.25) < 0.002
    assert abs(bench.dst_flops_per_launch(w, "fp64") - 2.841e9) < 0.001e9
    # 127^3 x 256 FP64: x and y in one slab launch each way around the fused
    # z launch: 3 launches for 6 products; BF16x3 folds every axis separately
    w3 = W.WORKLOADS["heat3d_127x256"]
    assert bench.dst_launch_mix(w3, "fp64") == (3, 6)
    assert bench.dst_launch_mix(w3, "bf16x3") == (6, 6)
    assert bench.dst_launch_mix(w3, "fp32") == (3, 6)
    assert bench.dst_path(w3, "bf16x3") == "fold"
    # every product on the third fold (the slab launch's x and y, the z
    # pass): 2560 of the two-level fold's 4064 multiply-adds per vector
    # (h = 64: 32^2 + 32^2 + 32 * 32 + 32 * 31)
    assert bench.fold3_slab(w3, "fp64") and not bench.fold3_slab(w3, "fp32")
    per = bench.dst_product_flops(w3, "fp64")
    assert per == 2.0 * 4064 * w3.n * (w3.m // w3.m1)
    expect = 6 * per * 2560 / 4064 / 3
    assert abs(bench.dst_flops_per_launch(w3, "fp64") / expect - 1) < 1e-12


def test_record_only_when_checking():
    class Fake:
        def cpu(self):
            raise AssertionError("copied although the checks are off")
    bench.record(None, {}, ("heat", "heat2d_255x256"), Fake())
    checks = []

    class Dev:
        def cpu(self):
            return self

        def numpy(self):
            return "u"
    bench.record(checks, {"x": 1}, ("cd", "cd2d_255x256"), Dev())
    assert checks == [({"x": 1}, ("cd", "cd2d_255x256"), "u")]
