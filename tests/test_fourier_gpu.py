"""Fourier-shift sub-pixel patch (shift theorem on the integer window) on the GPU
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from gpu_util import compare, custom_problem, dev, rel_l2, run_gpu, run_oracle, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(prob, **kw):
    torch_cuda()
    from paper_2510_20929_amd import Plan
    return Plan.for_problem(prob, **kw)


@pytest.mark.parametrize("N,M,E,loss", [(16, 1, 1, "amplitude"), (32, 2, 1, "poisson"), (64, 3, 2, "amplitude"),
                                        (128, 2, 1, "poisson"), (128, 1, 3, "amplitude")])
def test_fourier_shift_matches_oracle(N, M, E, loss):
    start, I = custom_problem(300 + N + M + E, N, M, E, 1, 3 * N, 60, loss=loss, subpixel="fourier",
                              weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads)
    compare(got, ref, grads, tag=f"fourier N={N} M={M} E={E} {loss}")
    assert got["flags"] == 0


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("recompute", [0, 1])
def test_fourier_shift_thread_layouts(variant, recompute):
    """Every thread layout, far fields stored or recomputed, on 16 workgroups (70 positions:
    four or five per workgroup, ragged tail)."""
    start, I = custom_problem(330 + variant, 128, 3, 1, 1, 400, 70, subpixel="fourier")
    grads = ("obj", "probe", "pos")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": variant, "recompute": recompute, "grid": 16}), start, I, grads)
    compare(got, ref, grads, tag=f"fourier variant={variant} recompute={recompute} grid=16")


def test_integer_positions_agree_with_bilinear():
    import dataclasses
    start, I = custom_problem(340, 64, 2, 1, 1, 200, 50)
    start = dataclasses.replace(start, positions=np.floor(start.positions).astype(np.float32))
    a = run_gpu(_plan(start), start, I, ("obj", "probe"))
    fs = dataclasses.replace(start, subpixel="fourier")
    b = run_gpu(_plan(fs), fs, I, ("obj", "probe"))
    for key in ("loss", "I_pred", "g_obj", "g_probe"):
        assert rel_l2(b[key], a[key]) <= 1e-5, key


@pytest.mark.parametrize("N,M,E,loss", [(32, 2, 1, "poisson"), (128, 1, 2, "amplitude"), (256, 2, 1, "poisson"),
                                        (512, 1, 2, "amplitude")])
def test_fourier_shift_per_step_form(N, M, E, loss):
    """The per-step form of the Fourier-shift patch (window transform, shift, inverse
    transform per position; adjoint: position gradient from the spectra, window gradient
    F^-1(conj(S) F g_o) scattered at the integer corner) against the oracle: with the
    PLAIN flag for on-chip frames, and as the only form of 256^2 and 512^2 plans."""
    start, I = custom_problem(350 + N + M, N, M, E, 1, 3 * N if N <= 128 else N + 96, 12, loss=loss,
                              subpixel="fourier", weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads, plain=N <= 128)
    compare(got, ref, grads, tag=f"fourier per-step N={N} M={M} E={E} {loss}")
    assert got["flags"] == 0


def test_fourier_shift_unsupported_forms():
    torch_cuda()
    from paper_2510_20929_amd import PtyhipError
    start, I = custom_problem(341, 32, 1, 1, 1, 100, 10, subpixel="fourier")
    plan = _plan(start)
    args = (dev(start.obj), dev(start.probe), dev(start.positions), dev(I))
    with pytest.raises(PtyhipError):
        plan.apply_A(args[0], args[1], args[2])
