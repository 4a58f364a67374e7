"""Probe-mode orthogonalisation on the GPU against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_util import FWD_TOL, case, custom_problem, dev, rel_l2, torch_cuda
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _run(prob):
    torch = torch_cuda()
    from paper_2510_20929_amd import Plan
    plan = Plan.for_problem(prob)
    out, powers = plan.orthogonalize_modes(dev(prob.probe))
    torch.cuda.synchronize()
    return plan, out, powers.cpu().numpy()


@pytest.mark.parametrize("which", ["c1", "c5", "opr", "m1", "m3", "m64"])
def test_orthogonalize_matches_oracle(which):
    if which == "c1":
        p, _ = case(1, H=400, K=10)
    elif which == "c5":
        p = W.perturb(W.make_config(5, K=10), 5)
    elif which == "opr":
        p, _ = custom_problem(61, 64, 2, 3, 1, 200, 10, weights="opr")
    elif which == "m1":
        p, _ = custom_problem(62, 32, 1, 1, 1, 80, 5)
    elif which == "m3":
        p, _ = custom_problem(63, 32, 3, 1, 1, 80, 5)
    else:
        rng = np.random.default_rng(64)
        U = (rng.normal(size=(1, 64, 16, 16)) + 1j * rng.normal(size=(1, 64, 16, 16))).astype(np.complex64)
        p = W.Problem("m64", np.ones((1, 40, 40), np.complex64), U, np.zeros((5, 2), np.float32), None, "amplitude")
    _, out, powers = _run(p)
    ref, lam = oracle.orthogonalize_modes(p.probe)
    e_out = rel_l2(out.cpu().numpy(), ref)
    e_pow = rel_l2(powers, lam)
    print(f"orthogonalize {which}: modes {e_out:.2e} powers {e_pow:.2e}", flush=True)
    assert e_out <= FWD_TOL and e_pow <= FWD_TOL


def test_orthogonalized_probe_keeps_the_loss():
    torch = torch_cuda()
    p, I = case(1, H=400, K=120)
    plan, out, _ = _run(p)
    obj, pos, Im = dev(p.obj), dev(p.positions), dev(I)
    l0 = float(plan.forward(obj, dev(p.probe), pos, Im)[0])
    l1 = float(plan.forward(obj, out, pos, Im)[0])
    assert abs(l1 - l0) <= FWD_TOL * abs(l0)
    X = out[0].reshape(p.M, -1).to(torch.complex128)
    G = (X.conj() @ X.T).cpu().numpy()
    off = np.abs(G - np.diag(np.diag(G))).max() / np.abs(np.diag(G)).max()
    assert off < 1e-5


def test_rejects_in_place():
    torch_cuda()
    from paper_2510_20929_amd import Plan, PtyhipError
    p, _ = custom_problem(65, 32, 2, 1, 1, 80, 5)
    plan = Plan.for_problem(p)
    pr = dev(p.probe)
    with pytest.raises(PtyhipError):
        plan.orthogonalize_modes(pr, out=pr)


def test_orthogonalize_degenerate_spectrum():
    """A Gram matrix with a repeated eigenvalue: the eigenmodes of the repeated value are
    not unique (any orthonormal basis of their span is correct), so the result is checked
    by what defines it: the new modes are orthogonal with the Gram eigenvalues as powers,
    the strongest mode matches the oracle (unique up to the phase convention), the pair
    spans the same subspace as the oracle's pair, the mode-summed intensity is unchanged
    at every pixel and so is the loss."""
    torch = torch_cuda()
    rng = np.random.default_rng(66)
    N, M = 32, 3
    B = rng.normal(size=(M, N * N)) + 1j * rng.normal(size=(M, N * N))
    Q, _ = np.linalg.qr(B.T)                                   # orthonormal columns
    base = (Q.T * np.sqrt([50.0, 20.0, 20.0])[:, None]).reshape(M, N, N)   # powers 50, 20, 20
    V, _ = np.linalg.qr(rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M)))
    U = np.einsum("jm,mab->jab", V, base)[None].astype(np.complex64)       # mixed: Gram not diagonal
    p = W.Problem("degenerate", np.ones((1, 3 * N, 3 * N), np.complex64), U,
                  rng.uniform(0, 2 * N - 2, size=(12, 2)).astype(np.float32), None, "amplitude")
    plan, out, powers = _run(p)
    got = out.cpu().numpy().astype(np.complex128)[0].reshape(M, -1)
    G = got.conj() @ got.T
    off = np.abs(G - np.diag(np.diag(G))).max() / np.abs(np.diag(G)).max()
    print(f"degenerate: off-diagonal {off:.2e}, powers {powers}", flush=True)
    assert off < 1e-5
    assert rel_l2(powers, [50.0, 20.0, 20.0]) <= 1e-5
    assert rel_l2(np.real(np.diag(G)), powers) <= 1e-5
    ref, lam = oracle.orthogonalize_modes(U)
    ref = ref[0].reshape(M, -1)
    assert rel_l2(got[0], ref[0]) <= 1e-5                     # the non-degenerate mode
    # the degenerate pair spans the oracle pair's subspace
    Qr, _ = np.linalg.qr(ref[1:].T)
    resid = got[1:].T - Qr @ (Qr.conj().T @ got[1:].T)
    assert np.linalg.norm(resid) <= 1e-5 * np.linalg.norm(got[1:])
    I0 = np.sum(np.abs(U[0].astype(np.complex128)) ** 2, axis=0)
    I1 = np.sum(np.abs(got.reshape(M, N, N)) ** 2, axis=0)
    assert rel_l2(I1, I0) <= 1e-5
    Im = rng.uniform(0, 50, size=(12, N, N)).astype(np.float32)
    l0 = float(plan.forward(dev(p.obj), dev(U), dev(p.positions), dev(Im))[0])
    l1 = float(plan.forward(dev(p.obj), out, dev(p.positions), dev(Im))[0])
    assert abs(l1 - l0) <= FWD_TOL * abs(l0)
