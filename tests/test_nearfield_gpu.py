"""Near-field (Fresnel to the detector) forward model, its gradients and the
det_lambda_z gradient on the GPU against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from gpu_util import compare, custom_problem, dev, run_gpu, run_oracle, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(prob, **kw):
    torch_cuda()
    from paper_2510_20929_amd import Plan
    return Plan.for_problem(prob, **kw)


def _lz(N):
    return (N / 2.0) ** 2 / 50.0   # Fresnel number 50


@pytest.mark.parametrize("N,M,E,loss", [(16, 1, 1, "amplitude"), (32, 2, 1, "poisson"), (64, 3, 2, "amplitude"),
                                        (128, 2, 1, "poisson")])
def test_near_field_matches_oracle(N, M, E, loss):
    start, I = custom_problem(200 + N + M, N, M, E, 1, 3 * N, 60, loss=loss, det_lambda_z=_lz(N),
                              weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos", "lambda_z") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start), start, I, grads)
    compare(got, ref, grads, tag=f"near N={N} M={M} E={E} {loss}")
    assert got["flags"] == 0


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_near_field_thread_layouts(variant):
    """Every thread layout of the near-field kernel on 16 workgroups (70 positions: four or
    five per workgroup, ragged tail)."""
    start, I = custom_problem(230 + variant, 128, 2, 1, 1, 400, 70, det_lambda_z=30.0)
    grads = ("obj", "probe", "lambda_z")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": variant, "grid": 16}), start, I, grads)
    compare(got, ref, grads, tag=f"near variant={variant} grid=16")


@pytest.mark.parametrize("N,M,E,loss", [(32, 2, 1, "poisson"), (128, 2, 2, "amplitude"), (256, 2, 1, "poisson"),
                                        (512, 1, 2, "amplitude")])
def test_near_field_per_step_form(N, M, E, loss):
    """The per-step form of the near field (F^-1 H F per mode, the loss in natural pixel
    order, the adjoint F^-1 conj(H) F) against the oracle: with the PLAIN flag for on-chip
    frames, and as the only form of 256^2 and 512^2 near-field plans (the four-step kernel
    models the far field), where the lambda-z gradient is refused."""
    torch = torch_cuda()
    from paper_2510_20929_amd import PtyhipError
    start, I = custom_problem(260 + N + M, N, M, E, 1, 3 * N if N <= 128 else N + 96, 12, loss=loss,
                              det_lambda_z=_lz(N), weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    plan = _plan(start)
    got = run_gpu(plan, start, I, grads, plain=N <= 128)
    compare(got, ref, grads, tag=f"near per-step N={N} M={M} E={E} {loss}")
    assert got["flags"] == 0
    if N > 128:
        w = None if start.weights is None else dev(start.weights)
        with pytest.raises(PtyhipError):
            plan.forward_adjoint(dev(start.obj), dev(start.probe), dev(start.positions), dev(I), weights=w,
                                 grads=("obj", "lambda_z"))


def test_near_field_zero_distance_and_errors():
    torch = torch_cuda()
    from paper_2510_20929_amd import PtyhipError
    start, I = custom_problem(240, 32, 2, 1, 1, 100, 30, det_lambda_z=0.0)
    ref = run_oracle(start, I, ("obj",))
    got = run_gpu(_plan(start), start, I, ("obj",))
    compare(got, ref, ("obj",), tag="near lz=0")
    plan = _plan(start)
    args = (dev(start.obj), dev(start.probe), dev(start.positions), dev(I))
    with pytest.raises(PtyhipError):
        plan.forward_adjoint(*args, grads=("obj", "lambda_z"), plain=True)   # the fused kernels compute dL/dlz
    with pytest.raises(PtyhipError):
        plan.apply_A(args[0], args[1], args[2])
    far, _ = custom_problem(241, 32, 1, 1, 1, 100, 10)
    fplan = _plan(far)
    with pytest.raises(PtyhipError):
        fplan.forward_adjoint(dev(far.obj), dev(far.probe), dev(far.positions),
                              torch.zeros((10, 32, 32), device="cuda"), grads=("lambda_z",))
