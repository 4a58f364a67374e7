"""The all-core timing harness of the oracle: worker processes over position shards."""
import numpy as np
import pytest

from oracle import timing
from synth import workloads as W


@pytest.mark.timeout(300)
def test_pool_rate_runs_shards():
    p = W.make_config(0, K=16)
    I_meas = np.ones((p.K, p.N, p.N))
    rate, done, wall = timing.pool_rate(p.obj, p.probe, p.positions, I_meas, workers=2, budget_s=0.3, chunk=4,
                                        loss=p.loss, grads=("obj", "probe"))
    assert done >= 2 * 4 and done % 4 == 0
    assert wall >= 0.3 and rate == pytest.approx(done / wall)


def test_host_workers_bounds():
    assert 1 <= timing.host_workers() <= 16
    assert timing.host_workers(cap=1) == 1
