"""The autotuner only times candidates that pass parity against the per-step form,
returns the fastest and caches it by architecture and shape."""
import json

import pytest

from gpu_util import case, custom_problem, dev, torch_cuda
from synth import workloads as W

pytestmark = pytest.mark.gpu


def test_tune_plan_and_cache(tmp_path):
    torch_cuda()
    from paper_2510_20929_amd import autotune
    p, I = case(1, H=320, K=60)
    shape = dict(N=p.N, M=p.M, E=p.E, S=p.S, H=p.H, W=p.W, loss=p.loss, eps=p.eps, lambda_z=p.lambda_z)
    cache = str(tmp_path / "cache.json")
    tune, rep = autotune.tune_plan(shape, dev(p.obj), dev(p.probe), dev(p.positions), dev(I), cache_path=cache,
                                   reps=3)
    timed = [c for c in rep["candidates"] if "ms" in c]
    assert timed and all("parity" not in c for c in timed)
    assert tune in [c["tune"] for c in timed]
    data = json.load(open(cache))
    assert rep["key"] in data and data[rep["key"]]["tune"] == tune
    tune2, rep2 = autotune.tune_plan(shape, dev(p.obj), dev(p.probe), dev(p.positions), dev(I), cache_path=cache)
    assert rep2["cached"] and tune2 == tune


def test_tune_batch():
    torch_cuda()
    from paper_2510_20929_amd import autotune
    import numpy as np
    from gpu_util import measured
    truths = W.make_batched_config(n_datasets=4, k_scale=0.02, seed=5)
    starts = [W.perturb(t, 3) for t in truths]
    tens = [(dev(s.obj), dev(s.probe), dev(s.positions), dev(measured(t, 4)), dev(s.weights))
            for s, t in zip(starts, truths)]
    choice, rep = autotune.tune_batch(starts, tens, grads=("obj", "probe", "pos", "weights"), reps=2,
                                      cache_path=None)
    timed = [c for c in rep["candidates"] if "ms" in c]
    assert timed and not any("parity" in c for c in rep["candidates"])
    # the choice is the fastest timed candidate (serial or concurrent classes at some
    # workgroup total, or one call per dataset)
    assert choice == min(timed, key=lambda c: c["ms"])["tune"]
