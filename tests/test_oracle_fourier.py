"""Pins of the oracle's Fourier-shift sub-pixel patch (shift theorem on the integer
window) and of the gradients through it (no GPU)."""
import math

import numpy as np
import pytest

import oracle


def test_integer_position_is_a_crop():
    rng = np.random.default_rng(0)
    Os = rng.normal(size=(20, 24)) + 1j * rng.normal(size=(20, 24))
    np.testing.assert_allclose(oracle.fourier_patch(Os, 3, 5, 0.0, 0.0, 8), Os[3:11, 5:13], atol=1e-13)


@pytest.mark.parametrize("u,v,fy,fx", [(1, 2, 0.3, 0.6), (-3, 1, 0.75, 0.1), (0, -2, 0.5, 0.0)])
def test_plane_wave_closed_form(u, v, fy, fx):
    """A window-periodic plane wave shifted by (fy, fx) is the same plane wave sampled
    at the shifted coordinates."""
    N, y0, x0 = 8, 2, 3
    y, x = np.mgrid[0:20, 0:20]
    Os = np.exp(2j * math.pi * (u * y + v * x) / N)
    yy, xx = np.mgrid[0:N, 0:N]
    expect = np.exp(2j * math.pi * (u * (y0 + fy + yy) + v * (x0 + fx + xx)) / N)
    np.testing.assert_allclose(oracle.fourier_patch(Os, y0, x0, fy, fx, N), expect, atol=1e-12)


def test_adjoint_identity_and_unitarity():
    rng = np.random.default_rng(1)
    N = 8
    Os = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    g = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    o = oracle.fourier_patch(Os, 4, 2, 0.37, 0.81, N)
    back = np.zeros_like(Os)
    oracle.fourier_scatter(back, g, 4, 2, 0.37, 0.81)
    assert abs(np.vdot(g, o) - np.vdot(back, Os)) < 1e-11 * abs(np.vdot(g, o))
    assert abs(np.linalg.norm(o) - np.linalg.norm(Os[4:12, 2:10])) < 1e-12 * np.linalg.norm(o)


def test_gradients_finite_difference():
    rng = np.random.default_rng(2)
    N, H, K = 8, 20, 3
    O = (np.exp(1j * rng.uniform(-0.5, 0.5, size=(1, H, H))) * rng.uniform(0.8, 1.0, size=(1, H, H)))
    U = rng.normal(size=(1, 2, N, N)) + 1j * rng.normal(size=(1, 2, N, N))
    pos = rng.uniform(0.5, H - N - 1.5, size=(K, 2))
    pos = np.floor(pos) + np.clip(pos - np.floor(pos), 0.1, 0.9)
    I = rng.uniform(0.5, 3.0, size=(K, N, N))
    out = oracle.forward_adjoint(O, U, pos, I, grads=("obj", "probe", "pos"), subpixel="fourier")
    h = 1e-6
    L = lambda o, u, r: oracle.forward(o, u, r, I, subpixel="fourier")[0]
    for name, g in (("obj", out["g_obj"]), ("probe", out["g_probe"])):
        base = O if name == "obj" else U
        d = rng.normal(size=base.shape) + 1j * rng.normal(size=base.shape)
        if name == "obj":
            fd = (L(O + h * d, U, pos) - L(O - h * d, U, pos)) / (2 * h)
        else:
            fd = (L(O, U + h * d, pos) - L(O, U - h * d, pos)) / (2 * h)
        assert abs(float(np.sum(np.real(np.conj(g) * d))) - fd) <= 1e-6 * abs(fd)
    d = rng.normal(size=pos.shape) * 0.1
    fd = (L(O, U, pos + h * d) - L(O, U, pos - h * d)) / (2 * h)
    assert abs(float(np.sum(out["g_pos"] * d)) - fd) <= 1e-6 * abs(fd)
