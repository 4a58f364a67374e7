"""Pins of the oracle's illumination map and scale-normalised gradients against closed
forms and independently written definitions (no GPU)."""
import numpy as np
import pytest

import oracle


def _ones_probe(N, M=1):
    U = np.zeros((1, M, N, N), dtype=np.complex128)
    U[0, 0] = 1.0
    return U


@pytest.mark.parametrize("fy,fx", [(0.0, 0.0), (0.25, 0.0), (0.0, 0.6), (0.3, 0.7)])
def test_constant_probe_closed_form(fy, fx):
    """|P|^2 = 1 on the whole frame: the illumination is the outer product of the 1D
    bilinear footprints (1 - f, 1, ..., 1, f) placed at the corner."""
    N, H, W, y0, x0 = 8, 20, 22, 5, 7
    ill = oracle.illumination(_ones_probe(N), np.array([[y0 + fy, x0 + fx]]), H, W)
    ry = np.zeros(H)
    ry[y0:y0 + N] = 1.0
    ry[y0] -= fy
    ry[y0 + N] += fy
    rx = np.zeros(W)
    rx[x0:x0 + N] = 1.0
    rx[x0] -= fx
    rx[x0 + N] += fx
    np.testing.assert_allclose(ill, np.outer(ry, rx), atol=1e-14)


def test_integer_positions_are_shifted_sums():
    rng = np.random.default_rng(0)
    N, M, H, W = 6, 3, 17, 19
    U = rng.normal(size=(1, M, N, N)) + 1j * rng.normal(size=(1, M, N, N))
    pos = np.array([[0, 0], [3, 5], [11, 13], [4, 4]], dtype=np.float64)
    ref = np.zeros((H, W))
    A = np.sum(np.abs(U[0]) ** 2, axis=0)
    for y, x in pos.astype(int):
        ref[y:y + N, x:x + N] += A
    np.testing.assert_allclose(oracle.illumination(U, pos, H, W), ref, rtol=1e-13)


def test_mass_conservation_with_opr_weights():
    rng = np.random.default_rng(1)
    N, M, E, K, H = 8, 2, 3, 5, 30
    U = rng.normal(size=(E, M, N, N)) + 1j * rng.normal(size=(E, M, N, N))
    w = rng.normal(size=(K, E))
    pos = rng.uniform(0, H - N - 2, size=(K, 2))
    tot = sum(np.sum(np.abs(np.tensordot(w[k], U, axes=(0, 0))) ** 2) for k in range(K))
    ill = oracle.illumination(U, pos, H, H, weights=w)
    assert abs(ill.sum() - tot) < 1e-10 * tot
    assert ill.min() >= 0.0


def test_weight_scaling_and_mode_mixing_invariance():
    rng = np.random.default_rng(2)
    N, M, K, H = 8, 3, 4, 24
    U = rng.normal(size=(1, M, N, N)) + 1j * rng.normal(size=(1, M, N, N))
    pos = rng.uniform(0, H - N - 2, size=(K, 2))
    base = oracle.illumination(U, pos, H, H)
    c = rng.uniform(0.5, 1.5, size=(K, 1))
    sep = sum(c[k, 0] ** 2 * oracle.illumination(U, pos[k:k + 1], H, H) for k in range(K))
    np.testing.assert_allclose(oracle.illumination(U, pos, H, H, weights=c), sep, rtol=1e-12)
    Q, _ = np.linalg.qr(rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M)))
    mixed = np.einsum("mn,enij->emij", Q, U)
    np.testing.assert_allclose(oracle.illumination(mixed, pos, H, H), base, rtol=1e-12)


def test_normalized_object_gradient_is_epie_form():
    """One position, one mode, amplitude loss: the normalised object gradient equals
    2 p* (psi - psi') / max|p|^2 with psi' the magnitude-updated exit wave, written here
    from the paper's description without the oracle's adjoint."""
    rng = np.random.default_rng(3)
    N, H = 8, 12
    O = np.exp(1j * rng.uniform(-0.5, 0.5, size=(1, H, H))) * rng.uniform(0.8, 1.0, size=(1, H, H))
    p = (rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)))
    U = p[None, None]
    I_meas = rng.uniform(0.5, 2.0, size=(1, N, N))
    out = oracle.forward_adjoint(O, U, np.array([[2.0, 3.0]]), I_meas, loss="amplitude", grads=("obj", "probe"))
    g_obj, g_probe = oracle.normalized_gradients(out["g_obj"], out["g_probe"], O, U, 1)
    o = O[0, 2:2 + N, 3:3 + N]
    psi = p * o
    Psi = np.fft.fft2(psi, norm="ortho")
    Im = np.fft.ifftshift(I_meas[0])
    psi_upd = np.fft.ifft2(np.sqrt(Im) * Psi / np.abs(Psi), norm="ortho")
    expect_o = 2.0 * np.conj(p) * (psi - psi_upd) / np.max(np.abs(p) ** 2)
    np.testing.assert_allclose(g_obj[0, 2:2 + N, 3:3 + N], expect_o, rtol=1e-10, atol=1e-12)
    mask = np.ones((H, H), bool)
    mask[2:2 + N, 3:3 + N] = False
    assert np.abs(g_obj[0][mask]).max() == 0.0
    expect_p = 2.0 * np.conj(o) * (psi - psi_upd) / np.max(np.abs(O) ** 2)
    np.testing.assert_allclose(g_probe[0, 0], expect_p, rtol=1e-10, atol=1e-12)


def test_probe_power_max_with_weights():
    rng = np.random.default_rng(4)
    U = rng.normal(size=(2, 2, 4, 4)) + 1j * rng.normal(size=(2, 2, 4, 4))
    w = np.array([[1.0, 0.0], [0.0, 2.0], [0.5, 0.5]])
    cand = [np.max(np.sum(np.abs(np.tensordot(w[k], U, axes=(0, 0))) ** 2, axis=0)) for k in range(3)]
    assert oracle.probe_power_max(U, 3, weights=w) == pytest.approx(max(cand), rel=1e-14)
    assert oracle.probe_power_max(U[:1], 3) == pytest.approx(np.max(np.sum(np.abs(U[0]) ** 2, axis=0)), rel=1e-14)
