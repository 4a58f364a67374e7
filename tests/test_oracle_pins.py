"""Pins of the FP64 oracle against facts it does not compute itself.

Each test checks the oracle against brute force, a closed form, an invariant or a
reduction to a simpler case, chosen so that a dropped term, a wrong sign or index,
or a transposed operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from synth import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
rng0 = np.random.default_rng(7)


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ----------------------------------------------------------------------------- FFT

@pytest.mark.parametrize("N", [4, 8, 16])
def test_fft_matches_bruteforce_dft(N):
    x = crandn(rng0, N, N)
    ref = np.zeros((N, N), complex)
    for ky in range(N):
        for kx in range(N):
            acc = 0j
            for y in range(N):
                for xx in range(N):
                    acc += x[y, xx] * complex(math.cos(-2 * math.pi * (ky * y + kx * xx) / N),
                                              math.sin(-2 * math.pi * (ky * y + kx * xx) / N))
            ref[ky, kx] = acc / N
    np.testing.assert_allclose(oracle.fft2u(x), ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.dft2_bruteforce(x), ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.ifft2u(oracle.fft2u(x)), x, atol=1e-12)


def test_plane_wave_golden():
    gold = json.load(open(os.path.join(GOLD, "plane_wave.json")))
    for case in gold["cases"]:
        N, u, v = case["N"], case["u"], case["v"]
        y, x = np.mgrid[0:N, 0:N]
        O = np.exp(2j * math.pi * (u * y + v * x) / N)
        U = np.ones((1, 1, N, N), complex)
        _, I = oracle.forward(O, U, np.zeros((1, 2)), np.ones((1, N, N)))
        by, bx = case["bright"]
        assert abs(I[0, by, bx] - case["value"]) < 1e-9
        I[0, by, bx] = 0.0
        assert np.abs(I).max() < 1e-9


def test_delta_object_flat_intensity():
    N = 16
    O = np.zeros((N, N), complex)
    O[0, 0] = 1.0
    _, I = oracle.forward(O, np.ones((1, 1, N, N)), np.zeros((1, 2)), np.ones((1, N, N)))
    np.testing.assert_allclose(I[0], np.full((N, N), 1.0 / N ** 2), atol=1e-14)


def test_parseval_per_frame_integer_positions():
    rng = np.random.default_rng(3)
    N, M = 16, 3
    O = crandn(rng, 40, 40)
    U = crandn(rng, 1, M, N, N)
    pos = np.array([[0, 0], [5, 11], [24, 3]], float)
    _, I = oracle.forward(O, U, pos, np.ones((3, N, N)))
    for k, (py, px) in enumerate(pos.astype(int)):
        crop = O[py:py + N, px:px + N]
        energy = sum(np.sum(np.abs(U[0, m] * crop) ** 2) for m in range(M))
        assert abs(I[k].sum() - energy) < 1e-9 * energy


# ----------------------------------------------------------------------------- propagator

def test_fresnel_gaussian_beam_closed_form():
    """Paraxial propagation of a Gaussian exp(-r^2/a^2) under exp(-i pi lz f^2):
    u_z = (pi a^2 / (pi a^2 + i lz)) exp(-pi r^2 / (pi a^2 + i lz))."""
    N, a, lz = 64, 4.0, 20.0
    c = N // 2
    y, x = np.mgrid[0:N, 0:N] - c
    r2 = x * x + y * y
    u0 = np.exp(-r2 / a ** 2)
    q = math.pi * a * a + 1j * lz
    expect = (math.pi * a * a / q) * np.exp(-math.pi * r2 / q)
    got = oracle.propagate(u0, oracle.fresnel_tf(N, lz))
    np.testing.assert_allclose(got, expect, atol=1e-10)


def test_propagator_group_and_unitarity():
    rng = np.random.default_rng(5)
    N = 16
    x = crandn(rng, N, N)
    h1, h2 = oracle.fresnel_tf(N, 3.0), oracle.fresnel_tf(N, 5.5)
    h12 = oracle.fresnel_tf(N, 8.5)
    np.testing.assert_allclose(oracle.propagate(oracle.propagate(x, h1), h2), oracle.propagate(x, h12), atol=1e-12)
    assert abs(np.linalg.norm(oracle.propagate(x, h1)) - np.linalg.norm(x)) < 1e-12
    np.testing.assert_allclose(oracle.propagate(x, oracle.fresnel_tf(N, 0.0)), x, atol=1e-12)


# ----------------------------------------------------------------------------- patches

def test_bilinear_reproduces_ramp_and_its_slope():
    rng = np.random.default_rng(11)
    H, N = 30, 8
    al, be, ga = crandn(rng, 3)
    yy, xx = np.mgrid[0:H, 0:H]
    O = al * yy + be * xx + ga
    for (ry, rx) in [(3.25, 7.5), (0.0, 0.9), (12.75, 0.0), (5.0, 5.0)]:
        y0, x0, fy, fx = oracle.split_position((ry, rx), N, H, H, True)
        o = oracle.extract_patch(O, y0, x0, fy, fx, N)
        i, j = np.mgrid[0:N, 0:N]
        np.testing.assert_allclose(o, al * (ry + i) + be * (rx + j) + ga, atol=1e-12)
        dy, dx = oracle.patch_derivatives(O, y0, x0, fy, fx, N)
        np.testing.assert_allclose(dy, np.full((N, N), al), atol=1e-12)
        np.testing.assert_allclose(dx, np.full((N, N), be), atol=1e-12)


def test_integer_position_is_a_crop_and_scatter_is_transpose():
    rng = np.random.default_rng(12)
    H, N = 24, 8
    O = crandn(rng, H, H)
    y0, x0, fy, fx = oracle.split_position((4.0, 9.0), N, H, H, False)
    np.testing.assert_array_equal(oracle.extract_patch(O, y0, x0, fy, fx, N), O[4:12, 9:17])
    for r in [(4.0, 9.0), (2.3, 7.8), (0.5, 0.0)]:
        y0, x0, fy, fx = oracle.split_position(r, N, H, H, False)
        g = crandn(rng, N, N)
        gO = np.zeros_like(O)
        oracle.scatter_patch(gO, g, y0, x0, fy, fx)
        lhs = np.vdot(oracle.extract_patch(O, y0, x0, fy, fx, N), g)
        rhs = np.vdot(O, gO)
        assert abs(lhs - rhs) < 1e-10 * abs(lhs)
        assert abs(gO.sum() - g.sum()) < 1e-10 * abs(g.sum())      # bilinear weights sum to one


def test_window_bounds():
    H, N = 20, 8
    # the last integer corner is valid without position gradients only
    oracle.split_position((12.0, 12.0), N, H, H, False)
    with pytest.raises(ValueError):
        oracle.split_position((12.0, 12.0), N, H, H, True)
    with pytest.raises(ValueError):
        oracle.split_position((12.5, 0.0), N, H, H, False)
    with pytest.raises(ValueError):
        oracle.split_position((-0.25, 3.0), N, H, H, False)
    oracle.split_position((11.5, 11.5), N, H, H, True)


# ----------------------------------------------------------------------------- loss

def test_one_pixel_golden():
    gold = json.load(open(os.path.join(GOLD, "one_pixel.json")))
    for case in gold["cases"]:
        p = complex(*case["p"])
        o = complex(*case["o"])
        out = oracle.forward_adjoint(np.array([[o]]), np.array([[[[p]]]]), np.zeros((1, 2)),
                                     np.array([[[case["I_meas"]]]]), loss=case["loss"], eps=case["eps"],
                                     grads=("obj", "probe"))
        assert abs(out["loss"] - case["L"]) < 1e-12
        assert abs(out["I_pred"][0, 0, 0] - case["I"]) < 1e-12
        assert abs(out["g_obj"][0, 0, 0] - complex(*case["g_obj"])) < 1e-12
        assert abs(out["g_probe"][0, 0, 0, 0] - complex(*case["g_probe"])) < 1e-12


def _small_problem(seed, N=16, M=2, E=1, S=1, K=3, H=28, lz=0.0):
    rng = np.random.default_rng(seed)
    O = (1.0 + 0.3 * crandn(rng, S, H, H)).astype(complex)
    U = crandn(rng, E, M, N, N)
    pos = rng.uniform(0.1, H - N - 1.2, size=(K, 2))
    w = rng.normal(1.0, 0.3, size=(K, E)) if E > 1 else None
    Im = rng.poisson(5.0, size=(K, N, N)).astype(float) + 0.5
    return O, U, pos, w, Im


def test_zero_loss_and_zero_gradient_at_truth():
    O, U, pos, w, _ = _small_problem(1, M=2, E=2, S=2, lz=2.0)
    _, I = oracle.forward(O, U, pos, np.ones((3, 16, 16)), weights=w, lambda_z=2.0)
    out = oracle.forward_adjoint(O, U, pos, I, weights=w, lambda_z=2.0, loss="amplitude",
                                 grads=("obj", "probe", "pos", "weights"))
    assert out["loss"] < 1e-25
    for key in ("g_obj", "g_probe", "g_pos", "g_weights"):
        assert np.abs(out[key]).max() < 1e-12
    out = oracle.forward_adjoint(O, U, pos, I, weights=w, lambda_z=2.0, loss="poisson", eps=0.0,
                                 grads=("obj", "probe", "pos", "weights"))
    for key in ("g_obj", "g_probe", "g_pos", "g_weights"):
        assert np.abs(out[key]).max() < 1e-10


def test_eq2_printed_gradient_is_half_of_ours():
    """Eq. (2) gives dL/d(conj o); the g convention (dL/dRe + i dL/dIm) is twice that."""
    rng = np.random.default_rng(21)
    N, H = 16, 24
    O = 1.0 + 0.3 * crandn(rng, H, H)
    U = crandn(rng, 1, 1, N, N)
    pos = np.array([[3.0, 5.0]])
    Im = rng.uniform(0.5, 9.0, size=(1, N, N))
    ours = oracle.patch_gradients(O, U, pos, Im, loss="amplitude", norm_count=1)[0, 0]
    eq2 = oracle.eq2_patch_gradient(O, U, pos, Im, K_norm=1)
    np.testing.assert_allclose(ours, 2.0 * eq2, rtol=1e-12, atol=1e-14)


# ----------------------------------------------------------------------------- finite differences

def _fd_check(f, x0, analytic, idx, h=1e-6, rtol=1e-6):
    """Central differences of the real scalar f along real coordinates idx of x0."""
    x0 = np.array(x0, dtype=float, copy=True)
    flat = x0.reshape(-1)
    an = analytic.reshape(-1)
    errs, scale = [], np.abs(an).max()
    for i in idx:
        old = flat[i]
        flat[i] = old + h
        fp = f(x0)
        flat[i] = old - h
        fm = f(x0)
        flat[i] = old
        errs.append(abs((fp - fm) / (2 * h) - an[i]))
    assert max(errs) <= rtol * max(scale, 1e-12) + 1e-9, (max(errs), scale)


@pytest.mark.parametrize("loss", ["amplitude", "poisson"])
@pytest.mark.parametrize("S,E,M", [(1, 1, 1), (1, 3, 2), (3, 2, 2)])
def test_finite_differences_every_gradient(loss, S, E, M):
    lz = 2.5 if S > 1 else 0.0
    O, U, pos, w, Im = _small_problem(100 + S * 10 + E, M=M, E=E, S=S, lz=lz)
    kw = dict(weights=w, loss=loss, eps=1e-3, lambda_z=lz)
    grads = ("obj", "probe", "pos") + (("weights",) if w is not None else ())
    out = oracle.forward_adjoint(O, U, pos, Im, grads=grads, **kw)
    rng = np.random.default_rng(99)

    def c2r(z):
        return np.stack([z.real, z.imag], axis=-1)

    def r2c(a):
        return a[..., 0] + 1j * a[..., 1]

    Or = c2r(O)
    _fd_check(lambda a: oracle.forward(r2c(a), U, pos, Im, **kw)[0], Or, c2r(out["g_obj"]),
              rng.choice(Or.size, 80, replace=False))
    Ur = c2r(U)
    _fd_check(lambda a: oracle.forward(O, r2c(a), pos, Im, **kw)[0], Ur, c2r(out["g_probe"]),
              rng.choice(Ur.size, 80, replace=False))
    _fd_check(lambda a: oracle.forward(O, U, a, Im, **kw)[0], pos, out["g_pos"], range(pos.size))
    if w is not None:
        _fd_check(lambda a: oracle.forward(O, U, pos, Im, **{**kw, "weights": a})[0], w,
                  out["g_weights"], range(w.size))


# ----------------------------------------------------------------------------- linear maps

@pytest.mark.parametrize("S,E", [(1, 1), (3, 2)])
def test_adjoint_identity(S, E):
    rng = np.random.default_rng(31 + S)
    lz = 1.7
    O, U, pos, w, _ = _small_problem(40 + S, M=2, E=E, S=S, lz=lz)
    A = oracle.apply_A(O, U, pos, weights=w, lambda_z=lz)
    Y = crandn(rng, *A.shape)
    gO, gU = oracle.apply_AH(Y, O, U, pos, weights=w, lambda_z=lz)
    # probe map (object fixed): A(U) is linear in U
    X = crandn(rng, *U.shape)
    lhs = np.vdot(oracle.apply_A(O, X, pos, weights=w, lambda_z=lz), Y)
    assert abs(lhs - np.vdot(X, gU)) < 1e-10 * abs(lhs)
    # each slice map (other slices and probe fixed)
    for s in range(S):
        Xo = O.copy()
        Xo[s] = crandn(rng, *O.shape[1:])
        lhs = np.vdot(oracle.apply_A(Xo, U, pos, weights=w, lambda_z=lz), Y)
        assert abs(lhs - np.vdot(Xo[s], gO[s])) < 1e-10 * abs(lhs)


def test_intensity_is_sum_of_mode_powers_of_A():
    O, U, pos, w, Im = _small_problem(50, M=3, E=2, S=2)
    A = oracle.apply_A(O, U, pos, weights=w, lambda_z=1.0)
    _, I = oracle.forward(O, U, pos, Im, weights=w, lambda_z=1.0)
    np.testing.assert_allclose(I, oracle.centre(np.sum(np.abs(A) ** 2, axis=1)), rtol=1e-12)


def test_multislice_zero_distance_is_single_slice_of_product():
    O, U, pos, _, Im = _small_problem(60, M=2, S=3)
    a = oracle.forward_adjoint(O, U, pos, Im, lambda_z=0.0, grads=())
    pos_int = np.floor(pos)          # integer positions: the patch of a product is the product of patches
    a = oracle.forward(O, U, pos_int, Im, lambda_z=0.0)
    b = oracle.forward(np.prod(O, axis=0), U, pos_int, Im)
    assert abs(a[0] - b[0]) < 1e-12 * abs(b[0])
    np.testing.assert_allclose(a[1], b[1], rtol=1e-11)


def test_opr_reductions_and_mode_mixing():
    rng = np.random.default_rng(70)
    O, U, pos, _, Im = _small_problem(70, M=3, E=1)
    base = oracle.forward_adjoint(O, U, pos, Im, grads=("obj", "probe"))
    w1 = oracle.forward_adjoint(O, U, pos, Im, weights=np.ones((3, 1)), grads=("obj", "probe"))
    assert abs(base["loss"] - w1["loss"]) < 1e-14
    np.testing.assert_allclose(base["g_obj"], w1["g_obj"], atol=1e-14)
    _, I = oracle.forward(O, U, pos, Im)
    _, I2 = oracle.forward(O, U, pos, Im, weights=np.full((3, 1), 1.7))
    np.testing.assert_allclose(I2, 1.7 ** 2 * I, rtol=1e-12)
    # unitary mixing of the incoherent modes leaves the intensity unchanged
    q, _ = np.linalg.qr(crandn(rng, 3, 3))
    Umix = np.einsum("ab,ebyx->eayx", q, U)
    _, I3 = oracle.forward(O, Umix, pos, Im)
    np.testing.assert_allclose(I3, I, rtol=1e-11)


def test_batched_equals_sum_of_single_positions_and_shards():
    O, U, pos, w, Im = _small_problem(80, M=2, E=2, K=5)
    kw = dict(weights=w, loss="poisson", grads=("obj", "probe", "pos", "weights"))
    full = oracle.forward_adjoint(O, U, pos, Im, **kw)
    acc = {k: 0.0 for k in ("loss", "g_obj", "g_probe")}
    for k in range(5):
        one = oracle.forward_adjoint(O, U, pos[k:k + 1], Im[k:k + 1], norm_count=5,
                                     **{**kw, "weights": w[k:k + 1]})
        for key in acc:
            acc[key] = acc[key] + one[key]
        np.testing.assert_allclose(one["g_pos"][0], full["g_pos"][k], rtol=1e-12)
        np.testing.assert_allclose(one["g_weights"][0], full["g_weights"][k], rtol=1e-12)
    assert abs(acc["loss"] - full["loss"]) < 1e-12 * full["loss"]
    np.testing.assert_allclose(acc["g_obj"], full["g_obj"], atol=1e-13)
    np.testing.assert_allclose(acc["g_probe"], full["g_probe"], atol=1e-13)


# ----------------------------------------------------------------------------- synthetic inputs

def test_synthetic_configs_shapes_and_bounds():
    for c, kw in [(0, {}), (1, {}), (2, dict(H=700, K=400)), (3, dict(H=400, K=200, S=2)), (5, {})]:
        p = W.make_config(c, **kw)
        assert p.positions.dtype == np.float32 and p.obj.dtype == np.complex64
        assert p.positions.min() >= 0
        ext = 1 if "pos" in p.grads else 0
        assert (p.positions[:, 0] + p.N + ext <= p.H).all() and (p.positions[:, 1] + p.N + ext <= p.W).all()
        q = W.perturb(p, 5)
        assert (q.positions[:, 0] + p.N + 1 <= p.H).all() and q.positions.min() >= 0
    p0 = W.make_config(0)
    assert p0.K == 625 and p0.N == 64 and p0.positions.max() == 192
    p1 = W.make_config(1)
    assert p1.K == 2000 and p1.M == 4 and p1.H == 1024
    pw = np.sum(np.abs(p1.probe[0].astype(complex)) ** 2, axis=(1, 2))
    np.testing.assert_allclose(pw / pw.sum(), [0.7, 0.15, 0.1, 0.05], rtol=1e-5)
    p5 = W.make_config(5)
    assert (p5.K, p5.M, p5.N, p5.H, p5.W) == (6732, 30, 128, 413, 535)
    U = p5.probe[0].reshape(30, -1).astype(complex)
    G = U.conj() @ U.T
    off = np.abs(G - np.diag(np.diag(G))).max() / np.abs(np.diag(G)).max()
    assert off < 1e-5  # orthogonal modes
    d = np.diag(G).real
    np.testing.assert_allclose(d[1:] / d[:-1], np.exp(-1.0 / 6.0), rtol=1e-4)  # exp(-j/6) powers
