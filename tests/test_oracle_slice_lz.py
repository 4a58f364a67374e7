"""Pins of the oracle's slice-spacing gradient dL/d(lambda z) of the multislice model (no
GPU). The slice spacing enters every slice-to-slice Fresnel propagator; the automatic-
differentiation reconstructor refines it (Reconstructors). The pins do not reuse the
oracle's gradient formula: central finite differences of the loss, the propagator
composition H(z) H(z) = H(2 z) (a constant middle slice turns three slices at z into two
at 2 z, so the gradients differ by exactly the factor 2), and the invariance of the far
field under a last propagation onto a constant slice (zero gradient)."""
import numpy as np
import pytest

import oracle


def _crandn(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def _problem(seed, N=16, M=2, E=1, S=3, K=3, H=28):
    rng = np.random.default_rng(seed)
    O = np.exp(1j * 0.4 * rng.normal(size=(S, H, H))) * (1.0 + 0.2 * rng.normal(size=(S, H, H)))
    U = _crandn(rng, E, M, N, N)
    pos = rng.uniform(0.1, H - N - 1.2, size=(K, 2))
    w = rng.normal(1.0, 0.3, size=(K, E)) if E > 1 else None
    Im = rng.poisson(5.0, size=(K, N, N)).astype(float) + 0.5
    return O, U, pos, w, Im


@pytest.mark.parametrize("loss", ["amplitude", "poisson"])
@pytest.mark.parametrize("S,E,M", [(2, 1, 1), (3, 3, 2), (4, 1, 3)])
def test_slice_lambda_z_finite_difference(loss, S, E, M):
    O, U, pos, w, Im = _problem(500 + 10 * S + E + M, M=M, E=E, S=S)
    lz, h = 3.7, 1e-5
    kw = dict(weights=w, loss=loss, eps=1e-3)
    g = oracle.forward_adjoint(O, U, pos, Im, lambda_z=lz, grads=("lambda_z",), **kw)["g_lambda_z"]
    lp, _ = oracle.forward(O, U, pos, Im, lambda_z=lz + h, **kw)
    lm, _ = oracle.forward(O, U, pos, Im, lambda_z=lz - h, **kw)
    fd = (lp - lm) / (2 * h)
    assert abs(fd) > 1e-6                      # the loss does depend on the spacing here
    assert abs(g - fd) <= 1e-6 * abs(fd), (g, fd)


def test_slice_lambda_z_with_other_gradients_and_normaliser():
    """Requesting the other gradients alongside, and a global normaliser, leaves the
    spacing gradient as the finite difference of the same (normalised) loss."""
    O, U, pos, w, Im = _problem(531, M=2, E=2, S=3)
    lz, h, kn = 1.9, 1e-5, 17.0
    kw = dict(weights=w, loss="amplitude", norm_count=kn)
    out = oracle.forward_adjoint(O, U, pos, Im, lambda_z=lz, grads=("obj", "probe", "pos", "weights", "lambda_z"),
                                 **kw)
    fd = (oracle.forward(O, U, pos, Im, lambda_z=lz + h, **kw)[0]
          - oracle.forward(O, U, pos, Im, lambda_z=lz - h, **kw)[0]) / (2 * h)
    assert abs(out["g_lambda_z"] - fd) <= 1e-6 * abs(fd)


def test_composition_doubles_the_gradient():
    """Three slices with a constant middle slice at spacing z equal two slices at 2 z
    (the middle transmission is the identity and H(z) H(z) = H(2 z)); the loss is then
    L3(z) = L2(2 z), so dL3/dz = 2 dL2/d(2z)."""
    O, U, pos, _, Im = _problem(540, M=2, S=3)
    O3 = O.copy()
    O3[1] = 1.0
    O2 = O[[0, 2]]
    z = 2.3
    l3, _ = oracle.forward(O3, U, pos, Im, lambda_z=z)
    l2, _ = oracle.forward(O2, U, pos, Im, lambda_z=2 * z)
    assert abs(l3 - l2) <= 1e-12 * abs(l2)
    g3 = oracle.forward_adjoint(O3, U, pos, Im, lambda_z=z, grads=("lambda_z",))["g_lambda_z"]
    g2 = oracle.forward_adjoint(O2, U, pos, Im, lambda_z=2 * z, grads=("lambda_z",))["g_lambda_z"]
    assert abs(g3 - 2.0 * g2) <= 1e-10 * abs(g3)


def test_propagation_onto_a_constant_last_slice_has_no_effect():
    """With a constant last slice c, the far field of a two-slice model is c H F chi_0:
    the propagator only multiplies each detector pixel by a unimodular factor, so the
    intensity, the loss and hence the spacing gradient do not depend on the spacing."""
    O, U, pos, _, Im = _problem(550, M=2, S=2)
    O[1] = 0.7 + 0.2j                      # constant transmission of the last slice
    g = oracle.forward_adjoint(O, U, pos, Im, lambda_z=4.1, grads=("lambda_z",))["g_lambda_z"]
    l = oracle.forward(O, U, pos, Im, lambda_z=4.1)[0]
    assert abs(g) <= 1e-12 * abs(l)


def test_lambda_z_gradient_needs_a_propagator():
    O, U, pos, _, Im = _problem(560, S=1)
    with pytest.raises(ValueError):
        oracle.forward_adjoint(O, U, pos, Im, grads=("lambda_z",))
    O3, U3, pos3, _, Im3 = _problem(561, S=2)
    with pytest.raises(ValueError):
        oracle.forward_adjoint(O3, U3, pos3, Im3, lambda_z=1.0, det_lambda_z=2.0, grads=("lambda_z",))
