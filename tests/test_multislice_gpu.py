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
