"""The linear maps through the C ABI: apply_A against the oracle, apply_AH against the
oracle, and the adjoint identity <A x, y> = <x, A^H y> evaluated on the GPU."""
import numpy as np
import pytest

import oracle
from gpu_util import custom_problem, dev, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    torch_cuda()


@pytest.mark.parametrize("N,M,E,S", [(64, 2, 1, 1), (128, 1, 3, 1), (32, 2, 1, 3), (256, 3, 2, 1)])
def test_apply_A_AH(N, M, E, S):
    torch = torch_cuda()
    from paper_2510_20929_amd import Plan
    p, _ = custom_problem(500 + N + E + S, N, M, E, S, N * 3, 40, lz=N / 8.0,
                          weights="opr" if E > 1 else None)
    plan = Plan.for_problem(p)
    w = None if p.weights is None else dev(p.weights)
    Psi = plan.apply_A(dev(p.obj), dev(p.probe), dev(p.positions), weights=w)
    ref = oracle.apply_A(p.obj, p.probe, p.positions, weights=p.weights, lambda_z=p.lambda_z)
    e_a = rel_l2(Psi.cpu().numpy(), ref)
    rng = np.random.default_rng(3)
    Y = (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)).astype(np.complex64)
    gO, gU = plan.apply_AH(dev(Y), dev(p.obj), dev(p.probe), dev(p.positions), weights=w)
    torch.cuda.synchronize()
    rO, rU = oracle.apply_AH(Y, p.obj, p.probe, p.positions, weights=p.weights, lambda_z=p.lambda_z)
    e_o, e_u = rel_l2(gO.cpu().numpy(), rO), rel_l2(gU.cpu().numpy(), rU)
    print(f"apply_A {e_a:.2e} apply_AH obj {e_o:.2e} probe {e_u:.2e}")
    assert e_a <= 1e-5 and e_o <= 1e-4 and e_u <= 1e-4
    # adjoint identity on the GPU for the probe map: <A(X), Y> = <X, A^H Y>
    X = (rng.standard_normal(p.probe.shape) + 1j * rng.standard_normal(p.probe.shape)).astype(np.complex64)
    AX = plan.apply_A(dev(p.obj), dev(X), dev(p.positions), weights=w).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(AX, Y.astype(np.complex128))
    rhs = np.vdot(X.astype(np.complex128), gU.cpu().numpy().astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)
    # and for the last slice of the object
    Xo = p.obj.copy()
    Xo[-1] = (rng.standard_normal(Xo.shape[1:]) + 1j * rng.standard_normal(Xo.shape[1:])).astype(np.complex64)
    AXo = plan.apply_A(dev(Xo), dev(p.probe), dev(p.positions), weights=w).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(AXo, Y.astype(np.complex128))
    rhs = np.vdot(Xo[-1].astype(np.complex128), gO.cpu().numpy()[-1].astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)
