"""Pins of the oracle's probe-mode orthogonalisation against orthogonality, invariance
of the incoherent sum and closed forms (no GPU)."""
import numpy as np

import oracle


def _rand(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def test_orthogonal_and_sorted_and_sum_preserved():
    rng = np.random.default_rng(0)
    U = _rand(rng, 3, 5, 8, 8)
    out, lam = oracle.orthogonalize_modes(U)
    X = out[0].reshape(5, -1)
    G = np.array([[np.sum(np.conj(X[i]) * X[j]) for j in range(5)] for i in range(5)])
    np.testing.assert_allclose(G, np.diag(lam), atol=1e-9 * lam.max())
    assert np.all(np.diff(lam) <= 0)
    w = rng.normal(size=3)
    before = np.sum(np.abs(np.tensordot(w, U, axes=(0, 0))) ** 2, axis=0)
    after = np.sum(np.abs(np.tensordot(w, out, axes=(0, 0))) ** 2, axis=0)
    np.testing.assert_allclose(after, before, rtol=1e-10)


def test_already_orthogonal_modes_are_only_reordered():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(_rand(rng, 36, 4))
    modes = (Q.T * np.array([1.0, 3.0, 2.0, 0.5])[:, None]).reshape(1, 4, 6, 6)
    out, lam = oracle.orthogonalize_modes(modes)
    np.testing.assert_allclose(lam, [9.0, 4.0, 1.0, 0.25], rtol=1e-12)
    np.testing.assert_allclose(out[0], modes[0][[1, 2, 0, 3]], atol=1e-12)


def test_two_mode_closed_form():
    """P1 = a f1, P2 = b f1 + c f2 with orthonormal f: Gram [[a^2, a b], [a b, b^2 + c^2]],
    eigenvalues (tr +- sqrt(tr^2 - 4 det)) / 2."""
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(_rand(rng, 25, 2))
    f1, f2 = Q[:, 0], Q[:, 1]
    a, b, c = 2.0, 0.7, 1.3
    U = np.stack([a * f1, b * f1 + c * f2]).reshape(1, 2, 5, 5)
    tr, det = a * a + b * b + c * c, (a * a) * (b * b + c * c) - (a * b) ** 2
    disc = np.sqrt(tr * tr - 4 * det)
    _, lam = oracle.orthogonalize_modes(U)
    np.testing.assert_allclose(lam, [(tr + disc) / 2, (tr - disc) / 2], rtol=1e-12)


def test_forward_model_unchanged():
    rng = np.random.default_rng(3)
    N, H = 8, 20
    O = np.exp(1j * rng.uniform(-0.5, 0.5, size=(1, H, H)))
    U = _rand(rng, 2, 3, N, N)
    w = rng.normal(size=(4, 2))
    pos = rng.uniform(0, H - N - 2, size=(4, 2))
    I = rng.uniform(0.5, 2.0, size=(4, N, N))
    l0, I0 = oracle.forward(O, U, pos, I, weights=w)
    out, _ = oracle.orthogonalize_modes(U)
    l1, I1 = oracle.forward(O, out, pos, I, weights=w)
    np.testing.assert_allclose(I1, I0, rtol=1e-10)
    assert abs(l1 - l0) <= 1e-10 * abs(l0)


def test_phase_convention():
    rng = np.random.default_rng(4)
    U = _rand(rng, 1, 3, 4, 4)
    out, lam = oracle.orthogonalize_modes(U)
    X = U[0].reshape(3, -1)
    # recover V from out = V^T X (least squares, X has full row rank)
    V = np.linalg.lstsq(X.T, out[0].reshape(3, -1).T, rcond=None)[0]
    for j in range(3):
        m = int(np.argmax(np.abs(V[:, j])))
        assert abs(V[m, j].imag) < 1e-10 and V[m, j].real > 0
