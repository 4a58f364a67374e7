"""Multislice forward/adjoint on the GPU vs the FP64 oracle (store and recompute of the
incident waves, and the per-step form)."""
import pytest

from gpu_util import case, compare, custom_problem, run_gpu, run_oracle, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    torch_cuda()


def _plan(prob, **kw):
    from paper_2510_20929_amd import Plan
    return Plan.for_problem(prob, **kw)


TUNES = {"store": None, "recompute": {"recompute": 1},
         "fused_small_ms_kernel<128,1024,0>-store": {"variant": 1, "grid": 16},
         "fused_small_ms_kernel<128,1024,0>-recompute": {"variant": 1, "recompute": 1, "grid": 16},
         "fused_small_ms_kernel<128,512,0>-grid16": {"variant": 0, "grid": 16},
         "bench-choice": "bench", "plain": None}


@pytest.mark.parametrize("form", list(TUNES))
def test_config3_reduced(form):
    """Config 3 structure (128^2, 2 modes, weak-phase slices, lambda z = 81.92 px^2,
    spiral scan, object/probe/position gradients) with 3 slices of 300^2 and 90 positions.
    The forms with 16 workgroups give each workgroup five or six positions (ragged tail);
    bench-choice is the instance the benchmark runs for the full 5000-position workload,
    also on 16 workgroups."""
    start, I = case(3, H=300, K=90, S=3)
    grads = ("obj", "probe", "pos")
    ref = run_oracle(start, I, grads)
    tune = TUNES[form]
    if tune == "bench":
        from gpu_util import bench_tune
        tune = dict(bench_tune(start, I, grads, key_K=5000), grid=16)
    plan = _plan(start, tune=tune)
    got = run_gpu(plan, start, I, grads, plain=(form == "plain"))
    compare(got, ref, grads, tag=f"c3 {form} {tune}")
    assert got["flags"] == 0


@pytest.mark.parametrize("N,S,M,E", [(32, 2, 1, 1), (64, 4, 2, 2)])
def test_multislice_small(N, S, M, E):
    start, I = custom_problem(300 + N + S, N, M, E, S, N * 3, 60, lz=N / 8.0,
                              weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    for plain in (False, True):
        got = run_gpu(_plan(start), start, I, grads, plain=plain)
        compare(got, ref, grads, tag=f"ms N={N} S={S} {'plain' if plain else 'fused'}")


@pytest.mark.parametrize("N,S,M,E,loss", [(256, 3, 2, 1, "amplitude"), (512, 2, 1, 2, "poisson")])
def test_multislice_large_frames_per_step_form(N, S, M, E, loss):
    """Multislice plans of 256^2 and 512^2 frames run the per-step form (the four-step
    kernel models one slice) against the oracle; the slice-spacing gradient is refused."""
    from paper_2510_20929_amd import PtyhipError
    from gpu_util import dev
    start, I = custom_problem(320 + N + S, N, M, E, S, N + 96, 6, lz=N / 8.0, loss=loss,
                              weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    plan = _plan(start)
    got = run_gpu(plan, start, I, grads)
    compare(got, ref, grads, tag=f"ms per-step N={N} S={S} M={M} E={E}")
    assert got["flags"] == 0
    w = None if start.weights is None else dev(start.weights)
    with pytest.raises(PtyhipError):
        plan.forward_adjoint(dev(start.obj), dev(start.probe), dev(start.positions), dev(I), weights=w,
                             grads=("obj", "lambda_z"))


@pytest.mark.parametrize("tune", [None, {"recompute": 1}, {"variant": 1, "grid": 16},
                                  {"variant": 1, "recompute": 1, "grid": 16}],
                         ids=["store", "recompute", "1024-store-grid16", "1024-recompute-grid16"])
def test_slice_spacing_gradient(tune):
    """dL/d(lambda z) of the slice spacing (with every other gradient) against the oracle,
    config 3 structure with 3 slices, stored or recomputed incident waves."""
    start, I = case(3, H=300, K=90, S=3)
    grads = ("obj", "probe", "pos", "lambda_z")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune=tune), start, I, grads)
    compare(got, ref, grads, tag=f"c3 slice lambda_z {tune}")
    assert got["flags"] == 0


@pytest.mark.parametrize("N,S,M,E,loss", [(32, 2, 1, 1, "poisson"), (64, 4, 2, 2, "amplitude")])
def test_slice_spacing_gradient_small(N, S, M, E, loss):
    start, I = custom_problem(330 + N + S, N, M, E, S, N * 3, 60, lz=N / 8.0, loss=loss,
                              weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "lambda_z") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads)
    compare(got, ref, grads, tag=f"ms lambda_z N={N} S={S} M={M} E={E}")


def test_slice_spacing_gradient_errors():
    import torch
    from paper_2510_20929_amd import PtyhipError
    from gpu_util import dev
    start, I = custom_problem(341, 32, 1, 1, 2, 100, 10, lz=3.0)
    plan = _plan(start)
    args = (dev(start.obj), dev(start.probe), dev(start.positions), dev(I))
    with pytest.raises(PtyhipError):
        plan.forward_adjoint(*args, grads=("obj", "lambda_z"), plain=True)   # fused form only
    single, I1 = custom_problem(342, 32, 1, 1, 1, 100, 10)
    with pytest.raises(PtyhipError):
        _plan(single).forward_adjoint(dev(single.obj), dev(single.probe), dev(single.positions), dev(I1),
                                      grads=("lambda_z",))                     # no propagator
    torch.cuda.synchronize()
