"""Configs 2, 3 and 4 at their full sizes, in the launch configuration the benchmark
times, checked against the FP64 oracle on sampled outputs it can compute piecewise:
  * per-position outputs (predicted intensity, position and weight gradients) of a
    sample of positions, from the oracle on just those positions with the global
    normaliser;
  * object-gradient tiles, from the oracle on the positions whose windows touch them;
and by properties at full size: the loss and probe gradient of the whole equal the sum
over shards (global normaliser), and the batched launch equals one call per dataset.
Measured intensities: the oracle's patterns at every position whose outputs are
compared (computed in parallel CPU processes), re-used for the others."""
import numpy as np
import pytest

import oracle
from gpu_util import FWD_TOL, GRAD_TOL, covering, dev, measured_sparse, rel_l2, run_oracle, torch_cuda
from synth import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

NAMES = {"obj": "g_obj", "probe": "g_probe", "pos": "g_pos", "weights": "g_weights"}


def _needed(start, ks, tiles):
    need = set(int(k) for k in ks)
    for (ty, tx, sz) in tiles:
        need.update(int(k) for k in covering(start, ty, tx, sz))
    return np.array(sorted(need))


def _full_launch(plan, start, I, grads):
    torch = torch_cuda()
    w = None if start.weights is None else dev(start.weights)
    ipred = torch.empty((start.K, start.N, start.N), dtype=torch.float32, device="cuda")
    args = (dev(start.obj), dev(start.probe), dev(start.positions), dev(I))
    out = plan.forward_adjoint(*args, weights=w, grads=grads, I_pred=ipred)
    torch.cuda.synchronize()
    assert plan.get_error() == 0
    return out, args, w


def _sampled_checks(start, I, grads, out, ks, tiles, tag):
    K = start.K
    # per-position outputs of sampled positions
    sub = start.subset(ks)
    ref = run_oracle(sub, I[ks], grads, norm_count=K)
    e = rel_l2(out["I_pred"][ks].cpu().numpy(), ref["I_pred"])
    print(f"{tag} I_pred[{len(ks)} sampled]: {e:.2e}", flush=True)
    assert e <= FWD_TOL
    for g in ("pos", "weights"):
        if g in grads:
            e = rel_l2(out[NAMES[g]][ks].cpu().numpy(), ref[NAMES[g]])
            print(f"{tag} {NAMES[g]}[sampled]: {e:.2e}", flush=True)
            assert e <= GRAD_TOL
    # object-gradient tiles
    g_obj = out["g_obj"]
    for (ty, tx, sz) in tiles:
        idx = covering(start, ty, tx, sz)
        r = run_oracle(start.subset(idx), I[idx], ("obj",), norm_count=K)
        got = g_obj[:, ty:ty + sz, tx:tx + sz].cpu().numpy()
        e = rel_l2(got, r["g_obj"][:, ty:ty + sz, tx:tx + sz])
        print(f"{tag} g_obj tile {(ty, tx, sz)} ({len(idx)} positions): {e:.2e}", flush=True)
        assert e <= GRAD_TOL


def _shard_sum(plan, args, w, grads, K, tag):
    torch = torch_cuda()
    o, u, r, m = args
    whole = plan.forward_adjoint(o, u, r, m, weights=w, grads=grads)
    half = K // 2
    acc = None
    for a, b in ((0, half), (half, K)):
        ws = None if w is None else w[a:b].contiguous()
        acc = plan.forward_adjoint(o, u, r[a:b].contiguous(), m[a:b].contiguous(), weights=ws,
                                   grads=("obj", "probe"), accumulate=acc is not None, out=None if acc is None else acc)
    torch.cuda.synchronize()
    for key in ("loss", "g_obj", "g_probe"):
        e = rel_l2(acc[key].cpu().numpy(), whole[key].cpu().numpy())
        print(f"{tag} shard-sum {key}: {e:.2e}", flush=True)
        assert e <= 1e-5


def test_config2_full_sampled():
    """Config 2 at full size (10000 positions, 8 eigenprobes of 256^2) on the instance the
    benchmark runs: the loss, the whole eigenprobe gradient, every position's weight and
    position gradients against the oracle summed over position shards (parallel CPU
    processes, global normaliser); predicted intensities of sampled positions and
    object-gradient tiles against the oracle on the positions that touch them."""
    torch_cuda()
    from gpu_util import bench_tune, run_oracle_sharded
    from paper_2510_20929_amd import Plan
    truth = W.make_config(2)
    start = W.perturb(truth, 5)
    rng = np.random.default_rng(7)
    ks = np.sort(rng.choice(start.K, 12, replace=False))
    tiles = [(1000, 1000, 8), (300, 1700, 8)]
    I = measured_sparse([truth], [_needed(start, ks, tiles)], [6])[0]
    grads = ("obj", "probe", "weights", "pos")
    tune = bench_tune(start, I, start.grads)
    plan = Plan.for_problem(start, norm_count=start.K, tune=tune)
    out, args, w = _full_launch(plan, start, I, grads)
    ref = run_oracle_sharded(start, I, ("probe", "weights", "pos"))
    e = abs(float(out["loss"].cpu()[0]) - ref["loss"]) / abs(ref["loss"])
    print(f"c2 full {tune} loss (all positions): {e:.2e}", flush=True)
    assert e <= FWD_TOL
    for key in ("g_probe", "g_weights", "g_pos"):
        e = rel_l2(out[key].cpu().numpy(), ref[key])
        print(f"c2 full {key} (all positions): {e:.2e}", flush=True)
        assert e <= GRAD_TOL
    _sampled_checks(start, I, grads, out, ks, tiles, "c2 full")
    _shard_sum(plan, args, w, grads, start.K, "c2 full")


C3_TILES = [(960, 960, 8), (400, 1500, 8)]


@pytest.fixture(scope="module")
def c3_inputs():
    truth = W.make_config(3)
    start = W.perturb(truth, 5)
    ks = np.sort(np.random.default_rng(8).choice(start.K, 12, replace=False))
    return start, measured_sparse([truth], [_needed(start, ks, C3_TILES)], [6])[0], ks


@pytest.mark.parametrize("recompute", [0, 1, "bench"], ids=["store", "recompute", "bench-choice"])
def test_config3_full_sampled(recompute, c3_inputs):
    torch_cuda()
    from gpu_util import bench_tune
    from paper_2510_20929_amd import Plan
    start, I, ks = c3_inputs
    grads = ("obj", "probe", "pos")
    tune = bench_tune(start, I, start.grads) if recompute == "bench" else {"recompute": recompute}
    plan = Plan.for_problem(start, norm_count=start.K, tune=tune)
    out, args, w = _full_launch(plan, start, I, grads)
    _sampled_checks(start, I, grads, out, ks, C3_TILES, f"c3 full {tune}")
    if recompute == 0:
        _shard_sum(plan, args, w, grads, start.K, "c3 full")


def test_config4_full_batched_vs_per_call_and_sampled():
    torch = torch_cuda()
    from paper_2510_20929_amd import Batch
    truths = W.make_batched_config()
    starts = [W.perturb(t, 3) for t in truths]
    # oracle samples: the first dataset of each frame size (3 positions and one 8 x 8 tile)
    rng = np.random.default_rng(9)
    picks, seen = {}, set()
    for i, s in enumerate(starts):
        if s.N in seen:
            continue
        seen.add(s.N)
        ty = int(s.positions[s.K // 2, 0])
        picks[i] = (np.sort(rng.choice(s.K, min(3, s.K), replace=False)), (ty, ty, 8))
    # whole-dataset oracle runs: the dataset with the fewest positions of each frame size
    whole = {}
    for i, s in enumerate(starts):
        if s.N not in whole or s.K < starts[whole[s.N]].K:
            whole[s.N] = i
    needs = [_needed(s, *((picks[i][0], [picks[i][1]]) if i in picks else (np.arange(min(8, s.K)), [])))
             for i, s in enumerate(starts)]
    Is = measured_sparse(truths, needs, [4 + i for i in range(len(truths))])
    grads = ("obj", "probe", "pos", "weights")
    b = Batch(starts)
    outs = [b.bind(i, dev(s.obj), dev(s.probe), dev(s.positions), dev(I), weights=dev(s.weights))
            for i, (s, I) in enumerate(zip(starts, Is))]
    b.launch(grads)
    torch.cuda.synchronize()
    assert b.get_error() == 0
    batched = [{k: v.clone() for k, v in o.items()} for o in outs]
    b.launch(grads, per_call=True)
    torch.cuda.synchronize()
    for i, (x, y) in enumerate(zip(batched, outs)):
        for key in ("loss", "g_obj", "g_probe", "g_pos", "g_weights"):
            e = rel_l2(x[key].cpu().numpy(), y[key].cpu().numpy())
            assert e <= 1e-5, f"dataset {i} {key}: batched vs per-call {e:.2e}"
    for i, (ks, (ty, tx, sz)) in picks.items():
        s = starts[i]
        ref = run_oracle(s.subset(ks), Is[i][ks], ("pos", "weights"), norm_count=s.K)
        for key in ("g_pos", "g_weights"):
            e = rel_l2(batched[i][key][ks].cpu().numpy(), ref[key])
            print(f"c4 dataset {i} (N={s.N}, K={s.K}) {key}[sampled]: {e:.2e}", flush=True)
            assert e <= GRAD_TOL
        idx = covering(s, ty, tx, sz)
        r = run_oracle(s.subset(idx), Is[i][idx], ("obj",), norm_count=s.K)
        e = rel_l2(batched[i]["g_obj"][:, ty:ty + sz, tx:tx + sz].cpu().numpy(), r["g_obj"][:, ty:ty + sz, tx:tx + sz])
        print(f"c4 dataset {i} g_obj tile ({len(idx)} positions): {e:.2e}", flush=True)
        assert e <= GRAD_TOL
    from gpu_util import run_oracle_sharded
    for N, i in sorted(whole.items()):
        s = starts[i]
        ref = run_oracle_sharded(s, Is[i], ("probe", "pos", "weights"))
        e = abs(float(batched[i]["loss"].cpu()[0]) - ref["loss"]) / abs(ref["loss"])
        print(f"c4 dataset {i} (N={N}, M={s.M}, K={s.K}) loss (all positions): {e:.2e}", flush=True)
        assert e <= FWD_TOL
        for key in ("g_probe", "g_pos", "g_weights"):
            e = rel_l2(batched[i][key].cpu().numpy(), ref[key])
            print(f"c4 dataset {i} (N={N}) {key} (all positions): {e:.2e}", flush=True)
            assert e <= GRAD_TOL
