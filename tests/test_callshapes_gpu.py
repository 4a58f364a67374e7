"""The paper's call shapes on the GPU against the FP64 oracle: minibatches of the
mode-heavy benchmark dataset (50 and 2000 positions per call, 30 modes), the supplement's
speed-benchmark shape (15 modes, 3 OPR eigenprobes, 128^2 and 512^2 frames, 16 positions
per call), each on the instance the benchmark runs for that call shape; and graph replay
of repeated calls (same tensors, K and flags) against direct calls."""
import numpy as np
import pytest

from gpu_util import bench_tune, case, compare, dev, measured, rel_l2, run_gpu, run_oracle, torch_cuda
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _plan(prob, **kw):
    torch_cuda()
    from paper_2510_20929_amd import Plan
    return Plan.for_problem(prob, **kw)


@pytest.mark.parametrize("B", [50, 2000])
def test_config5_minibatch_call(B):
    """One minibatch call of config 5 (30 modes of 128^2, 413 x 535 object) with the
    benchmark's tuned instance for B positions per call; at B = 2000 the call takes 96
    positions on 24 workgroups (several positions per workgroup, ragged tail)."""
    K = 50 if B == 50 else 96
    start, I = case(5, K=K)
    grads = start.grads
    tune = dict(bench_tune(start, I, grads, key_K=B))
    if B == 2000:
        tune["grid"] = 24
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune=tune), start, I, grads)
    compare(got, ref, grads, tag=f"c5 minibatch B={B} {tune}")
    assert got["flags"] == 0


@pytest.mark.parametrize("N", [128, 512])
def test_config6_supplement_shape(N):
    """Config 6 (15 modes, 3 OPR eigenprobes with per-position weights, amplitude loss,
    object/eigenprobe/weight gradients) with 16 positions per call, the supplement's batch
    size, on the benchmark's tuned instance (staged eigenprobe gradients)."""
    truth = W.make_config(6, N=N, K=16)
    start = W.perturb(truth, 5)
    I = measured(truth, 6)
    grads = ("obj", "probe", "weights")
    tune = bench_tune(start, I, start.grads, key_K=16)
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune=tune), start, I, grads)
    compare(got, ref, grads, tag=f"c6 N={N} {tune}")
    assert got["flags"] == 0


def test_config6_several_positions_per_workgroup():
    """Config 6 at 128^2 with 40 positions on 8 workgroups: staged eigenprobe gradients
    from workgroups that take five positions each."""
    truth = W.make_config(6, N=128, K=40)
    start = W.perturb(truth, 7)
    I = measured(truth, 8)
    grads = ("obj", "probe", "weights", "pos")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": 4, "recompute": 1, "grid": 8}), start, I, grads)
    compare(got, ref, grads, tag="c6 grid=8")


def test_graph_replay_matches_direct_calls():
    """Minibatch loop with graph replay on: every replay of a captured call equals the
    direct call bitwise; new data behind the same tensors is picked up by the replay; the
    ragged last minibatch is its own graph."""
    torch = torch_cuda()
    start, I = case(1, H=400, K=130)
    grads = ("obj", "probe", "pos")
    B = 48
    obj, probe, pos, meas = dev(start.obj), dev(start.probe), dev(start.positions), dev(I)
    calls = [(pos[a:a + B], meas[a:a + B]) for a in range(0, start.K, B)]
    direct = _plan(start, max_positions=B)
    ref = [direct.forward_adjoint(obj, probe, p, m, grads=grads) for p, m in calls]
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in r.items()} for r in ref]
    plan = _plan(start, max_positions=B)
    plan.set_graphs(True)
    outs = [plan.forward_adjoint(obj, probe, p, m, grads=grads) for p, m in calls]   # captures
    for rep in range(3):
        for (p, m), o in zip(calls, outs):
            plan.forward_adjoint(obj, probe, p, m, grads=grads, out=o)              # replays
        torch.cuda.synchronize()
        for r, o in zip(ref, outs):
            for key in ("loss", "g_obj", "g_probe", "g_pos"):
                assert torch.equal(r[key], o[key]), (rep, key)
    # new object values behind the same tensor: the replay computes with them
    obj.mul_(1.03)
    new_ref = [direct.forward_adjoint(obj, probe, p, m, grads=grads) for p, m in calls]
    for (p, m), o in zip(calls, outs):
        plan.forward_adjoint(obj, probe, p, m, grads=grads, out=o)
    torch.cuda.synchronize()
    for r, o in zip(new_ref, outs):
        for key in ("loss", "g_obj", "g_probe", "g_pos"):
            assert torch.equal(r[key], o[key]), key
    assert plan.get_error() == 0
    plan.set_graphs(False)


@pytest.mark.parametrize("M,E,G,N,loss", [(4, 1, 2, 128, "poisson"), (4, 1, 4, 128, "amplitude"),
                                          (15, 3, 4, 128, "amplitude"), (15, 3, 15, 64, "poisson"),
                                          (3, 2, 3, 32, "amplitude")])
@pytest.mark.parametrize("variant", [0, 4])
def test_mode_split_form(M, E, G, N, loss, variant):
    """The mode-split form (each position's modes in G groups, three launches) against the
    oracle, with eigenprobe weights or without, several groups of unequal size, every
    gradient, on 8 workgroups (several items per workgroup)."""
    from gpu_util import custom_problem
    start, I = custom_problem(700 + M + E + G + N, N, M, E, 1, N * 3, 20, loss=loss,
                              weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": variant, "mode_groups": G, "grid": 8}), start, I, grads)
    compare(got, ref, grads, tag=f"split M={M} E={E} G={G} N={N} variant={variant}")
    assert got["flags"] == 0


@pytest.mark.parametrize("M,E,G,N,loss,variant", [(3, 1, 3, 256, "poisson", 0), (4, 2, 2, 256, "amplitude", 1),
                                                  (5, 3, 2, 512, "amplitude", 0), (3, 1, 3, 512, "poisson", 1)])
def test_mode_split_form_fourstep(M, E, G, N, loss, variant):
    """The mode-split form of the four-step kernel (256^2, 512^2 frames) against the
    oracle: groups of one or several modes (unequal sizes for M = 5, G = 2), eigenprobe
    weights or none, every gradient, both thread layouts, on 6 workgroups so that each
    takes several (position, group) items."""
    from gpu_util import custom_problem
    start, I = custom_problem(760 + M + E + G + N, N, M, E, 1, N + 96, 9, loss=loss,
                              weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": variant, "mode_groups": G, "grid": 6}), start, I, grads)
    compare(got, ref, grads, tag=f"split four-step M={M} E={E} G={G} N={N} variant={variant}")
    assert got["flags"] == 0


@pytest.mark.parametrize("N,H", [(64, 200), (256, 360)])
def test_mode_split_forward_errors_and_accumulate(N, H):
    """Mode-split form (on-chip and four-step frames): the forward call alone (loss and
    predicted intensities), a position whose window leaves the object (latched and
    dropped, the rest exact), and two shards accumulated with the global normaliser equal
    to the whole."""
    torch = torch_cuda()
    import oracle
    from gpu_util import custom_problem
    start, I = custom_problem(731, N, 6, 1, 1, H, 24 if N <= 128 else 10, loss="poisson")
    tune = {"mode_groups": 3, "grid": 8}
    plan = _plan(start, tune=tune)
    o, u, r, m = dev(start.obj), dev(start.probe), dev(start.positions), dev(I)
    ipred = torch.zeros((start.K, N, N), dtype=torch.float32, device="cuda")
    loss = plan.forward(o, u, r, m, I_pred=ipred)
    torch.cuda.synchronize()
    ref_l, ref_I = oracle.forward(start.obj, start.probe, start.positions, I, loss=start.loss, eps=start.eps)
    compare({"loss": float(loss.cpu()[0]), "I_pred": ipred.cpu().numpy()}, {"loss": ref_l, "I_pred": ref_I}, (),
            tag="split forward")
    # one position outside the object
    bad = start.positions.copy()
    bad[5] = (H - 10.0, 3.0)
    rb = dev(bad)
    out = plan.forward_adjoint(o, u, rb, m, grads=("obj", "probe", "pos"))
    torch.cuda.synchronize()
    assert plan.get_error() & 1
    plan.clear_error()
    keep = np.array([k for k in range(start.K) if k != 5])
    ref = run_oracle(start.subset(keep), I[keep], ("obj", "probe", "pos"), norm_count=start.K)
    got = {k: v.cpu().numpy() for k, v in out.items()}
    assert rel_l2(got["g_obj"], ref["g_obj"]) <= 1e-4
    assert rel_l2(got["g_probe"], ref["g_probe"]) <= 1e-4
    assert rel_l2(np.delete(got["g_pos"], 5, axis=0), ref["g_pos"]) <= 1e-4
    assert np.all(got["g_pos"][5] == 0)
    # shards with the global normaliser add up to the whole
    sp = _plan(start, tune=tune, norm_count=start.K)
    whole = sp.forward_adjoint(o, u, r, m, grads=("obj", "probe"))
    acc = None
    for a_, b_ in ((0, 7), (7, start.K)):
        acc = sp.forward_adjoint(o, u, r[a_:b_].contiguous(), m[a_:b_].contiguous(), grads=("obj", "probe"),
                                 accumulate=acc is not None, out=None if acc is None else acc)
    torch.cuda.synchronize()
    for key in ("loss", "g_obj", "g_probe"):
        assert rel_l2(acc[key].cpu().numpy(), whole[key].cpu().numpy()) <= 1e-5, key
