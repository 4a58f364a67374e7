"""Config 1 at its full size (1024^2 object, 4 x 128^2 modes, 2000 positions) against
the oracle's full loss and gradients, on the kernel instance the benchmark times (the
autotuner's cached choice for these sources, looked up as bench.py does) and on the
fixed instances it chooses between; and the data-parallel shard-sum identity (gradients
of shards with the global normaliser add up to the whole).

With 2000 positions over one persistent workgroup per CU every workgroup takes several
positions, so the per-workgroup probe-gradient accumulation across positions and the
ragged tail of the persistent loop are part of what is compared."""
import numpy as np
import pytest

from gpu_util import bench_tune, case, compare, dev, kernel_instance, rel_l2, run_gpu, run_oracle, torch_cuda

pytestmark = pytest.mark.gpu

GRADS = ("obj", "probe", "pos")


@pytest.fixture(scope="module")
def c1():
    torch_cuda()
    start, I = case(1)
    return start, I, run_oracle(start, I, GRADS)


@pytest.mark.parametrize("tune", [
    "bench",
    {"variant": 4, "recompute": 1},
    {"variant": 4, "recompute": 0},
    {"variant": 1, "recompute": 1},
    {"variant": 0, "recompute": 0},
    {"variant": 5, "recompute": 1},
    {"variant": 6, "recompute": 1},
], ids=["bench-choice", "fused_small_kernel<128,1024,1,true,false>-recompute",
        "fused_small_kernel<128,1024,1,true,false>-store", "fused_small_kernel<128,1024,1,false,false>-recompute",
        "fused_small_kernel<128,512,1,false,false>-store", "fused_small_lds_kernel<128,1024,1,false>",
        "fused_small_lds_kernel<128,1024,1,true>"])
def test_config1_full_parity(c1, tune):
    from paper_2510_20929_amd import Plan
    start, I, ref = c1
    if tune == "bench":
        tune = bench_tune(start, I, GRADS)
    plan = Plan.for_problem(start, tune=tune)
    info = plan.info()
    assert info["grid"] < start.K
    name = kernel_instance(start, tune, info["threads"])
    got = run_gpu(plan, start, I, GRADS)
    compare(got, ref, GRADS, tag=f"c1 full {name} {tune} grid={info['grid']}")
    assert got["flags"] == 0


def test_config1_shard_sum(c1):
    torch = torch_cuda()
    from paper_2510_20929_amd import Plan
    start, I, _ = c1
    K = start.K
    plan = Plan.for_problem(start, norm_count=K)
    o, u, r, m = dev(start.obj), dev(start.probe), dev(start.positions), dev(I)
    whole = plan.forward_adjoint(o, u, r, m, grads=GRADS)
    shards = None
    bounds = [0, 333, 1000, 1001, 1700, K]
    for a, b in zip(bounds[:-1], bounds[1:]):
        part = plan.forward_adjoint(o, u, r[a:b].contiguous(), m[a:b].contiguous(), grads=("obj", "probe"),
                                    accumulate=shards is not None, out=None if shards is None else shards)
        shards = part
    torch.cuda.synchronize()
    for key in ("loss", "g_obj", "g_probe"):
        e = rel_l2(shards[key].cpu().numpy(), whole[key].cpu().numpy())
        print(f"shard-sum {key}: {e:.2e}")
        assert e <= 1e-5
