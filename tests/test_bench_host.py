"""Host-side checks of the figures bench.py derives (no GPU): the algorithmic work per
pattern, the per-call packing bound of uneven datasets, the refusal of several GPUs,
and the kernel names the bench line reports."""
import math
import subprocess
import sys
import types

import pytest

import bench
from synth import workloads as W


def test_algorithmic_flops_per_pattern():
    """Config 1: four modes, one slice -> 8 transforms of 5 N^2 log2 N^2 flops; config 3
    (8 slices, 2 modes): 2 + 4 (S - 1) = 30 transforms per mode."""
    p1 = W.make_config(1, K=16)
    flops, byts = bench.algorithmic(p1)
    assert flops == 8 * 5 * 128 * 128 * 14
    assert byts > 4 * 128 * 128
    p3 = W.make_config(3, K=4, H=400)
    assert bench.algorithmic(p3)[0] == 2 * 30 * 5 * 128 * 128 * 14


def test_packing_bound_hand_example():
    """Two datasets on 4 workgroups: 5 positions of cost c (2 rounds, 8 slots) and 4
    positions of cost 2c (1 round, 4 slots): work 5c + 8c = 13c, slots 8c + 8c = 16c."""
    def prob(N, M, K):
        return types.SimpleNamespace(N=N, M=M, K=K)
    c = 64 * 64 * math.log2(64 * 64)
    r = bench.packing_bound([prob(64, 1, 5), prob(64, 2, 4)], 4)
    assert r["per_call_occupancy"] == pytest.approx(13 * c / (16 * c))
    assert r["perfect_packing_gain"] == pytest.approx(16 / 13)
    # a dataset that fills whole rounds packs perfectly
    assert bench.packing_bound([prob(128, 3, 512)], 256)["per_call_occupancy"] == pytest.approx(1.0)


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_kernel_names_of_the_mode_split_form():
    plan = types.SimpleNamespace(info=lambda: {"threads": 1024})
    p128 = types.SimpleNamespace(N=128, M=15, S=1, loss="amplitude")
    p512 = types.SimpleNamespace(N=512, M=15, S=1, loss="amplitude")
    assert bench.kernel_name(plan, p128, {"mode_groups": 15}).startswith("split_forward/loss/adjoint_kernel<128, 1024>")
    assert bench.kernel_name(plan, p512, {"mode_groups": 15}).startswith("split_big_kernel<512, 1024, 1/2>")
    assert bench.kernel_name(plan, p512, {"variant": 0}) == "fused_big_kernel<512, 1024, 0>"
    p1 = types.SimpleNamespace(N=128, M=4, S=1, loss="poisson")
    assert bench.kernel_name(plan, p1, {"variant": 4}) == "fused_small_kernel<128, 1024, 1, true, false>"
    # the LDS-resident layouts
    assert bench.kernel_name(plan, p1, {"variant": 5}) == "fused_small_lds_kernel<128, 1024, 1, false>"
    assert bench.kernel_name(plan, p1, {"variant": 6}) == "fused_small_lds_kernel<128, 1024, 1, true>"
    assert bench.kernel_name(plan, p128, {"variant": 5, "mode_groups": 15}).startswith(
        "split_forward/loss/adjoint_lds_kernel<128, 1024>")
    p3 = types.SimpleNamespace(N=128, M=2, S=8, loss="amplitude")
    assert bench.kernel_name(plan, p3, {"variant": 5}) == "fused_small_lds_ms_kernel<128, 1024, 0>"
