"""GPU forward/adjoint vs the FP64 oracle on identical seeded inputs, through the C ABI.

Sizes are chosen so that the oracle finishes in seconds while the launches still span
several persistent rounds (K > number of workgroups) with a ragged tail."""
import numpy as np
import pytest

import oracle
from gpu_util import case, compare, custom_problem, dev, run_gpu, run_oracle, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    torch_cuda()


def _plan(prob, **kw):
    torch_cuda()
    from paper_2510_20929_amd import Plan
    return Plan.for_problem(prob, **kw)


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_config0_full(plain):
    """Config 0 at its full size: 256^2 object, 64^2 probe, 625 integer raster positions."""
    start, I = case(0)
    grads = ("obj", "probe")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads, plain=plain)
    compare(got, ref, grads, tag=f"c0 {'plain' if plain else 'fused'}")
    assert got["flags"] == 0


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_config1_reduced(plain):
    """Config 1 structure (128^2, 4 Hermite-Gauss modes, Poisson, sub-pixel spiral,
    object/probe/position gradients) on a 400^2 object with 300 positions."""
    start, I = case(1, H=400, K=300)
    grads = ("obj", "probe", "pos")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads, plain=plain)
    compare(got, ref, grads, tag=f"c1 {'plain' if plain else 'fused'}")
    assert got["flags"] == 0


@pytest.mark.parametrize("N,M,E", [(16, 1, 1), (32, 2, 3), (64, 3, 2), (128, 1, 4), (256, 3, 2)])
@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_opr_and_modes(N, M, E, plain):
    """Eigenprobes with per-position weights, several modes, every gradient."""
    start, I = custom_problem(100 + N + M + E, N, M, E, 1, N * 3, 70, loss="poisson" if M > 1 else "amplitude",
                              weights="opr")
    grads = ("obj", "probe", "pos", "weights")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads, plain=plain)
    compare(got, ref, grads, tag=f"opr N={N} M={M} E={E} {'plain' if plain else 'fused'}")


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_amplitude_weights_single_eigenprobe(plain):
    """Per-position probe amplitude (E = 1 with weights), as in the batched workload."""
    start, I = custom_problem(7, 64, 2, 1, 1, 200, 90, weights="amp")
    grads = ("obj", "probe", "pos", "weights")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads, plain=plain)
    compare(got, ref, grads, tag=f"amp-weights {'plain' if plain else 'fused'}")


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_config2_reduced(plain):
    """Config 2 structure (256^2 frames, 8 orthogonalised eigenprobes, per-position OPR
    weights, jittered raster, amplitude loss) on a 700^2 object with 300 positions."""
    start, I = case(2, H=700, K=300)
    grads = ("obj", "probe", "weights", "pos")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads, plain=plain)
    compare(got, ref, grads, tag=f"c2 {'plain' if plain else 'fused'}")
    assert got["flags"] == 0


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_frame512(plain):
    start, I = custom_problem(512, 512, 2, 1, 1, 700, 14, loss="poisson", weights="amp")
    grads = ("obj", "probe", "pos", "weights")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads, plain=plain)
    compare(got, ref, grads, tag=f"N=512 {'plain' if plain else 'fused'}")


@pytest.mark.parametrize("N,M,E", [(64, 2, 1), (256, 1, 3), (256, 3, 1), (512, 2, 1)])
def test_forward_only(N, M, E):
    """The forward call alone (loss and predicted intensities; no adjoint) against the
    oracle, on the on-chip and the four-step frames, one and several modes."""
    torch = torch_cuda()
    start, I = custom_problem(300 + N + M + E, N, M, E, 1, N * 2 + 40, 12, loss="poisson" if M > 1 else "amplitude",
                              weights="opr" if E > 1 else None)
    plan = _plan(start)
    w = None if start.weights is None else dev(start.weights)
    ipred = torch.zeros((start.K, N, N), dtype=torch.float32, device="cuda")
    loss = plan.forward(dev(start.obj), dev(start.probe), dev(start.positions), dev(I), weights=w, I_pred=ipred)
    torch.cuda.synchronize()
    ref_l, ref_I = oracle.forward(start.obj, start.probe, start.positions, I, weights=start.weights, loss=start.loss,
                                  eps=start.eps)
    got = {"loss": float(loss.cpu()[0]), "I_pred": ipred.cpu().numpy()}
    compare(got, {"loss": ref_l, "I_pred": ref_I}, (), tag=f"forward N={N} M={M} E={E}")
    assert plan.get_error() == 0


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("recompute", [0, 1])
@pytest.mark.parametrize("N", [64, 128])
def test_fused_variants(N, variant, recompute):
    """Every thread layout of the on-chip fused kernel (scratch- or register-resident
    patch), storing or recomputing the far fields, against the oracle, on a grid of 16
    workgroups: each workgroup takes five or six of the 90 positions (ragged tail), so
    its probe-gradient accumulator and the patch-gradient frames carry over from one
    position to the next. Four modes at 128^2 (the benchmark's shape), three at 64^2."""
    M = 4 if N == 128 else 3
    start, I = custom_problem(300 + N + 10 * variant + recompute, N, M, 2, 1, N * 3, 90, loss="poisson",
                              weights="opr")
    grads = ("obj", "probe", "pos", "weights")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": variant, "recompute": recompute, "grid": 16}), start, I, grads)
    compare(got, ref, grads, tag=f"N={N} M={M} variant={variant} recompute={recompute} grid=16")
    assert got["flags"] == 0


@pytest.mark.parametrize("recompute", [0, 1])
def test_fused_variants_single_eigenprobe(recompute):
    """The benchmark's headline instance (128^2, 1024 threads, patch in registers, patch
    gradient in scratch) with one unweighted eigenprobe and four modes, Poisson loss, on
    16 workgroups with a ragged tail (the weight-free probe loops of the headline workload)."""
    start, I = custom_problem(377 + recompute, 128, 4, 1, 1, 400, 75, loss="poisson")
    grads = ("obj", "probe", "pos")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": 4, "recompute": recompute, "grid": 16}), start, I, grads)
    compare(got, ref, grads, tag=f"headline layout recompute={recompute} grid=16")
    assert got["flags"] == 0


@pytest.mark.parametrize("N,E", [(256, 2), (512, 1)])
@pytest.mark.parametrize("variant", [0, 1])
def test_fourstep_layouts(N, E, variant):
    """Both layouts of the four-step fused kernel (one or two workgroups per CU), on a
    grid of 16 workgroups so that 40 positions take several persistent rounds with a
    ragged tail; staged eigenprobe gradients (E = 2) and per-workgroup accumulation
    (per-position amplitudes, E = 1)."""
    start, I = custom_problem(900 + N + E + variant, N, 2, E, 1, N * 2 + 60, 40, loss="poisson",
                              weights="opr" if E > 1 else "amp")
    grads = ("obj", "probe", "pos", "weights")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": variant, "grid": 16}), start, I, grads)
    compare(got, ref, grads, tag=f"four-step N={N} E={E} variant={variant}")
    assert got["flags"] == 0


@pytest.mark.parametrize("N,E", [(128, 2), (256, 3), (512, 1)])
def test_fused_bitwise_reproducible(N, E):
    """Two identical fused calls give bitwise-identical loss and gradients: the on-chip
    and four-step kernels, the per-workgroup and staged probe reductions, the window
    gather and the FP64 partial sums all add in a fixed order (no atomics)."""
    start, I = custom_problem(950 + N + E, N, 2, E, 1, N * 2 + 60, 24, loss="poisson",
                              weights="opr" if E > 1 else "amp")
    grads = ("obj", "probe", "pos", "weights")
    plan = _plan(start)
    a = run_gpu(plan, start, I, grads)
    b = run_gpu(plan, start, I, grads)
    assert a["flags"] == 0 and b["flags"] == 0
    for key in ("loss", "I_pred", "g_obj", "g_probe", "g_pos", "g_weights"):
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_config5_mode_heavy(plain):
    """Config 5 structure (30 probe modes of 128^2, 413 x 535 object, raster with sub-pixel
    offsets, amplitude loss) on its full object and probe with 48 positions."""
    start, I = case(5, K=48)
    grads = ("obj", "probe", "pos")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads, plain=plain)
    compare(got, ref, grads, tag=f"c5 {'plain' if plain else 'fused'}")
    assert got["flags"] == 0


@pytest.mark.parametrize("which", ["bench-choice", "fused_small_kernel<128,1024,0,true,false>-recompute"])
def test_config5_tuned_instance(which):
    """Config 5 (30 modes) on the instance the benchmark runs for its full 6732-position
    workload (the autotuner's cached choice) and on the 1024-thread register-patch layout
    with recomputed far fields, on 16 workgroups so that each takes three of the 48
    positions."""
    from gpu_util import bench_tune
    start, I = case(5, K=48)
    grads = ("obj", "probe", "pos")
    if which == "bench-choice":
        tune = dict(bench_tune(start, I, grads, key_K=6732))
    else:
        tune = {"variant": 4, "recompute": 1}
    tune["grid"] = 16
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune=tune), start, I, grads)
    compare(got, ref, grads, tag=f"c5 {which} {tune}")
    assert got["flags"] == 0


@pytest.mark.parametrize("N,M,variant", [(128, 4, 4), (128, 4, 1), (64, 2, 0), (256, 2, 0), (512, 1, 0)])
def test_probe_stage_single_eigenprobe(N, M, variant):
    """Probe gradients staged per position (tune probe_stage) with one unweighted
    eigenprobe, on 16 workgroups (several positions each), against the oracle."""
    start, I = custom_problem(960 + N + M, N, M, 1, 1, N * 2 + 60, 40, loss="poisson")
    grads = ("obj", "probe", "pos")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": variant, "recompute": 1, "grid": 16, "probe_stage": 1}), start, I,
                  grads)
    compare(got, ref, grads, tag=f"probe_stage N={N} M={M} variant={variant}")
    assert got["flags"] == 0
