"""Batched uneven reconstructions (config 4 structure, reduced): the captured persistent
launch against one call per dataset and against the FP64 oracle; graph replay is
deterministic; rebinding a dataset's buffers keeps the captured graph valid."""
import numpy as np
import pytest

import oracle
from gpu_util import compare, dev, measured, rel_l2, torch_cuda
from synth import workloads as W

pytestmark = pytest.mark.gpu
GRADS = ("obj", "probe", "pos", "weights")


@pytest.fixture(scope="module")
def batch_case():
    torch_cuda()
    truths = W.make_batched_config(n_datasets=8, k_scale=0.02, seed=5)
    assert sorted({p.N for p in truths}) == [64, 128, 256, 512]
    starts = [W.perturb(t, 40 + i) for i, t in enumerate(truths)]
    meas = [measured(t, 60 + i) for i, t in enumerate(truths)]
    return starts, meas


def _tensors(p, I):
    return dev(p.obj), dev(p.probe), dev(p.positions), dev(I), dev(p.weights)


def _np(out):
    return {k: (float(v[0]) if k == "loss" else v.cpu().numpy()) for k, v in out.items()}


def test_batched_graph_vs_per_call_and_oracle(batch_case):
    torch = torch_cuda()
    from paper_2510_20929_amd import Batch
    starts, meas = batch_case
    b = Batch(starts)
    outs = [b.bind(i, *_tensors(p, I)[:4], weights=_tensors(p, I)[4]) for i, (p, I) in enumerate(zip(starts, meas))]
    b.launch(GRADS)
    torch.cuda.synchronize()
    got = [_np(o) for o in outs]
    assert b.get_error() == 0
    pc = Batch(starts)
    pouts = [pc.bind(i, *_tensors(p, I)[:4], weights=_tensors(p, I)[4]) for i, (p, I) in enumerate(zip(starts, meas))]
    pc.launch(GRADS, per_call=True)
    torch.cuda.synchronize()
    for i, (p, I) in enumerate(zip(starts, meas)):
        per_call = _np(pouts[i])
        for k in ("g_obj", "g_probe", "g_pos", "g_weights"):
            assert rel_l2(got[i][k], per_call[k]) <= 1e-5, (i, k)
        ref = oracle.forward_adjoint(p.obj, p.probe, p.positions, I, weights=p.weights, loss=p.loss, grads=GRADS)
        compare(got[i], ref, GRADS, tag=f"batched {p.name} N={p.N} M={p.M} K={p.K}")


def test_graph_replay_is_deterministic_and_survives_rebinding(batch_case):
    torch = torch_cuda()
    from paper_2510_20929_amd import Batch
    starts, meas = batch_case
    b = Batch(starts)
    ts = [_tensors(p, I) for p, I in zip(starts, meas)]
    outs = [b.bind(i, *t[:4], weights=t[4]) for i, t in enumerate(ts)]
    b.launch(GRADS)
    torch.cuda.synchronize()
    first = [_np(o) for o in outs]
    b.launch(GRADS)  # replay of the captured graph
    torch.cuda.synchronize()
    second = [_np(o) for o in outs]
    for a, c in zip(first, second):
        for k in a:
            assert np.array_equal(np.asarray(a[k]), np.asarray(c[k])), k
    # rebind dataset 0 to a new object buffer and new outputs; the graph is replayed
    j = 0
    new_obj = (ts[j][0] * 1.05).contiguous()
    out_j = b.bind(j, new_obj, *ts[j][1:4], weights=ts[j][4])
    b.launch(GRADS)
    torch.cuda.synchronize()
    p, I = starts[j], meas[j]
    ref = oracle.forward_adjoint(new_obj.cpu().numpy(), p.probe, p.positions, I, weights=p.weights, loss=p.loss,
                                 grads=GRADS)
    compare(_np(out_j), ref, GRADS, tag="rebound")


def test_batched_per_step_mode(batch_case):
    torch = torch_cuda()
    from paper_2510_20929_amd import Batch
    starts, meas = batch_case
    sub = [0, 3, 6]
    b = Batch([starts[i] for i in sub])
    outs = [b.bind(j, *_tensors(starts[i], meas[i])[:4], weights=_tensors(starts[i], meas[i])[4])
            for j, i in enumerate(sub)]
    b.launch(GRADS, plain=True)
    torch.cuda.synchronize()
    for j, i in enumerate(sub):
        p, I = starts[i], meas[i]
        ref = oracle.forward_adjoint(p.obj, p.probe, p.positions, I, weights=p.weights, loss=p.loss, grads=GRADS)
        compare(_np(outs[j]), ref, GRADS, tag=f"batched plain {p.name}")


def test_batched_small_grid_vs_oracle(batch_case):
    """The batched launch on 8 workgroups per frame-size class (split among the class's
    datasets by work): the larger datasets give each of their workgroups several
    positions (ragged tails), so the per-workgroup probe-gradient accumulation of each
    class's body is compared with the oracle."""
    torch = torch_cuda()
    from paper_2510_20929_amd import Batch
    starts, meas = batch_case
    b = Batch(starts, tune={"grid": 8})
    outs = [b.bind(i, *_tensors(p, I)[:4], weights=_tensors(p, I)[4]) for i, (p, I) in enumerate(zip(starts, meas))]
    b.launch(GRADS)
    torch.cuda.synchronize()
    assert b.get_error() == 0
    for i, (p, I) in enumerate(zip(starts, meas)):
        ref = oracle.forward_adjoint(p.obj, p.probe, p.positions, I, weights=p.weights, loss=p.loss, grads=GRADS)
        compare(_np(outs[i]), ref, GRADS, tag=f"batched grid=8 {p.name} N={p.N} M={p.M} K={p.K}")


@pytest.mark.parametrize("tune", [{"variant": 1}, {"variant": 1, "grid": 24}], ids=["concurrent", "concurrent-24"])
def test_batched_concurrent_classes_vs_oracle(batch_case, tune):
    """The frame-size classes as concurrent graph branches (launches sharing the CUs by
    work), replayed twice: both replays against the oracle and bitwise equal."""
    torch = torch_cuda()
    from paper_2510_20929_amd import Batch
    starts, meas = batch_case
    b = Batch(starts, tune=tune)
    outs = [b.bind(i, *_tensors(p, I)[:4], weights=_tensors(p, I)[4]) for i, (p, I) in enumerate(zip(starts, meas))]
    b.launch(GRADS)
    torch.cuda.synchronize()
    first = [_np(o) for o in outs]
    b.launch(GRADS)
    torch.cuda.synchronize()
    assert b.get_error() == 0
    for i, (p, I) in enumerate(zip(starts, meas)):
        again = _np(outs[i])
        for k in first[i]:
            assert np.array_equal(np.asarray(first[i][k]), np.asarray(again[k])), k
        ref = oracle.forward_adjoint(p.obj, p.probe, p.positions, I, weights=p.weights, loss=p.loss, grads=GRADS)
        compare(first[i], ref, GRADS, tag=f"batched {tune} {p.name} N={p.N} M={p.M} K={p.K}")
