"""Pins of the oracle's near-field (Fresnel-to-detector) model and its gradients (no GPU)."""
import numpy as np
import pytest

import oracle


def _problem(seed, N=8, H=20, M=2, K=3):
    rng = np.random.default_rng(seed)
    O = (np.exp(1j * rng.uniform(-0.6, 0.6, size=(1, H, H))) * rng.uniform(0.7, 1.0, size=(1, H, H)))
    U = rng.normal(size=(1, M, N, N)) + 1j * rng.normal(size=(1, M, N, N))
    pos = rng.uniform(0, H - N - 2, size=(K, 2))
    I = rng.uniform(0.5, 4.0, size=(K, N, N))
    return O, U, pos, I


def test_zero_distance_is_exit_wave_intensity():
    O, U, _, I = _problem(0, K=1)
    N = U.shape[-1]
    pos = np.array([[3.0, 5.0]])
    _, Ip = oracle.forward(O, U, pos, I, det_lambda_z=0.0)
    chi = U[0] * O[0, 3:3 + N, 5:5 + N][None]
    np.testing.assert_allclose(Ip[0], np.sum(np.abs(chi) ** 2, axis=0), rtol=1e-12)


def test_energy_is_conserved():
    O, U, pos, I = _problem(1)
    _, I0 = oracle.forward(O, U, pos, I, det_lambda_z=0.0)
    _, I1 = oracle.forward(O, U, pos, I, det_lambda_z=23.7)
    np.testing.assert_allclose(I1.sum(axis=(1, 2)), I0.sum(axis=(1, 2)), rtol=1e-12)
    assert np.abs(I1 - I0).max() > 1e-3 * I0.max()  # the pattern itself changes


@pytest.mark.parametrize("loss", ["amplitude", "poisson"])
def test_lambda_z_gradient_finite_difference(loss):
    O, U, pos, I = _problem(2)
    lz, h = 17.3, 1e-5
    g = oracle.forward_adjoint(O, U, pos, I, loss=loss, grads=("lambda_z",), det_lambda_z=lz)["g_lambda_z"]
    lp, _ = oracle.forward(O, U, pos, I, loss=loss, det_lambda_z=lz + h)
    lm, _ = oracle.forward(O, U, pos, I, loss=loss, det_lambda_z=lz - h)
    fd = (lp - lm) / (2 * h)
    assert abs(g - fd) <= 1e-6 * max(abs(fd), 1e-12)


def test_object_and_probe_gradients_finite_difference():
    O, U, pos, I = _problem(3)
    lz = 11.0
    out = oracle.forward_adjoint(O, U, pos, I, grads=("obj", "probe", "pos"), det_lambda_z=lz)
    rng = np.random.default_rng(4)
    h = 1e-6
    for name, base, g in (("obj", O, out["g_obj"]), ("probe", U, out["g_probe"])):
        d = rng.normal(size=base.shape) + 1j * rng.normal(size=base.shape)
        def L(x):
            if name == "obj":
                return oracle.forward(x, U, pos, I, det_lambda_z=lz)[0]
            return oracle.forward(O, x, pos, I, det_lambda_z=lz)[0]
        fd = (L(base + h * d) - L(base - h * d)) / (2 * h)
        an = float(np.sum(np.real(np.conj(g) * d)))
        assert abs(an - fd) <= 1e-6 * abs(fd)
    dpos = rng.normal(size=pos.shape)
    fd = (oracle.forward(O, U, pos + h * dpos, I, det_lambda_z=lz)[0]
          - oracle.forward(O, U, pos - h * dpos, I, det_lambda_z=lz)[0]) / (2 * h)
    an = float(np.sum(out["g_pos"] * dpos))
    assert abs(an - fd) <= 1e-6 * abs(fd)


def test_far_field_only_rejects_lambda_z_gradient():
    O, U, pos, I = _problem(5)
    with pytest.raises(ValueError):
        oracle.forward_adjoint(O, U, pos, I, grads=("lambda_z",))
