"""FP64 CPU oracle for the far-field ptychographic forward model and its exact adjoint.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or execute
this module: only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use it. It shares no code with the GPU library.

What it computes (arxiv 2510.20929, Pty-Chi):
  * the forward model of Sec. 2.1 (patch extraction, exit wave psi = p * o, free-space
    propagation to the far field, several incoherent probe modes, scan-point-specific
    probes from orthogonal probe relaxation, multislice), giving the predicted
    intensity I_p = F(o, p, Lambda) of Eq. (4);
  * the Gaussian (magnitude MSE) loss of Eq. (1), and a Poisson negative
    log-likelihood (the paper names no formula; reading below);
  * the gradients of that loss: the object-patch gradient has the form of Eq. (2)
    (conjugate probe times the difference between the magnitude-updated and the
    forward exit wave), extended to the probe, the OPR weights, the scan positions
    and every multislice slice by the chain rule.

Readings where the paper is silent (each is a documented choice, not a derivation):
  * FFT: unitary ("ortho") 2D DFT with kernel exp(-2 pi i k.n / N).
  * Detector arrays (measured and predicted intensity) are DC-centred (fftshift).
  * Position r = (y, x) is the frame's top-left corner in object pixels; the patch is
    the bilinear interpolation of the object at the fractional offset; taps whose
    weight is exactly zero are not read.  The window is N x N, widened by one row
    (column) when the fraction is non-zero or position gradients are requested.
    A window outside the object raises ValueError.
  * Gradient convention: g = dL/dRe z + i dL/dIm z (twice the conjugate Wirtinger
    derivative; 2 x the value printed in Eq. (2)).
  * Loss normaliser 1 / (K_norm N^2); K_norm defaults to the number of positions.
  * Poisson: l = I - I_meas ln(I + eps), eps in photons, constants dropped.
  * Amplitude loss: the ratio I_meas / I floors I at 1e-30.
  * OPR: P_{k,m} = sum_e w_{k,e} U_{e,m} with real w, applied to every mode.
  * Multislice: transmit, then propagate by H = exp(-i pi lz (fy^2 + fx^2)) (fy, fx in
    cycles per pixel), S - 1 propagations, the last exit wave goes to the far field;
    every slice uses the same position.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

AMP_FLOOR = 1e-30


# ----------------------------------------------------------------------------- transforms

def fft2u(x: np.ndarray) -> np.ndarray:
    """Unitary 2D DFT over the last two axes (forward kernel exp(-2 pi i k n / N))."""
    return np.fft.fft2(x, norm="ortho")


def ifft2u(x: np.ndarray) -> np.ndarray:
    """Inverse of ``fft2u`` (its adjoint, since the transform is unitary)."""
    return np.fft.ifft2(x, norm="ortho")


def dft2_bruteforce(x: np.ndarray) -> np.ndarray:
    """The same unitary 2D DFT written as explicit sums over a DFT matrix (slow pin)."""
    n = x.shape[-1]
    k = np.arange(n)
    F = np.exp(-2j * math.pi * np.outer(k, k) / n) / math.sqrt(n)
    return F @ x.astype(np.complex128) @ F.T


def centre(a: np.ndarray) -> np.ndarray:
    """Unshifted detector layout -> DC-centred layout."""
    return np.fft.fftshift(a, axes=(-2, -1))


def uncentre(a: np.ndarray) -> np.ndarray:
    """DC-centred detector layout -> unshifted layout."""
    return np.fft.ifftshift(a, axes=(-2, -1))


def fresnel_tf(N: int, lambda_z: float) -> np.ndarray:
    """Free-space transfer function exp(-i pi lz (fy^2 + fx^2)) on the unshifted grid."""
    f = np.fft.fftfreq(N)
    fy, fx = np.meshgrid(f, f, indexing="ij")
    return np.exp(-1j * math.pi * lambda_z * (fy * fy + fx * fx))


def propagate(x: np.ndarray, tf: np.ndarray) -> np.ndarray:
    """Slice-to-slice propagation: inverse DFT of the transfer function times the DFT."""
    return ifft2u(tf * fft2u(x))


def propagate_adjoint(g: np.ndarray, tf: np.ndarray) -> np.ndarray:
    return ifft2u(np.conj(tf) * fft2u(g))


# ----------------------------------------------------------------------------- patches

def split_position(r: Sequence[float], N: int, H: int, W: int, want_pos: bool):
    """Integer corner and fraction of one scan position, with the window bounds check."""
    ry, rx = float(r[0]), float(r[1])
    y0, x0 = int(math.floor(ry)), int(math.floor(rx))
    fy, fx = ry - y0, rx - x0
    ey = 1 if (fy > 0.0 or want_pos) else 0
    ex = 1 if (fx > 0.0 or want_pos) else 0
    if y0 < 0 or x0 < 0 or y0 + N - 1 + ey > H - 1 or x0 + N - 1 + ex > W - 1:
        raise ValueError(f"scan window at {(ry, rx)} leaves the {H}x{W} object")
    return y0, x0, fy, fx


def _taps(fy: float, fx: float):
    """Bilinear taps (a, b, weight) with the zero-weight ones dropped."""
    out = []
    for a, wa in ((0, 1.0 - fy), (1, fy)):
        if wa == 0.0:
            continue
        for b, wb in ((0, 1.0 - fx), (1, fx)):
            if wb == 0.0:
                continue
            out.append((a, b, wa * wb))
    return out


def extract_patch(Os: np.ndarray, y0: int, x0: int, fy: float, fx: float, N: int) -> np.ndarray:
    """Object patch at a sub-pixel position: bilinear interpolation of one slice."""
    o = np.zeros((N, N), dtype=np.complex128)
    for a, b, w in _taps(fy, fx):
        o += w * Os[y0 + a:y0 + a + N, x0 + b:x0 + b + N]
    return o


def scatter_patch(gOs: np.ndarray, g: np.ndarray, y0: int, x0: int, fy: float, fx: float) -> None:
    """Transpose of ``extract_patch``: add the patch gradient back into the slice."""
    N = g.shape[-1]
    for a, b, w in _taps(fy, fx):
        gOs[y0 + a:y0 + a + N, x0 + b:x0 + b + N] += w * g


def patch_derivatives(Os: np.ndarray, y0: int, x0: int, fy: float, fx: float, N: int):
    """d(patch)/dy and d(patch)/dx of the bilinear patch (right derivative at integers)."""
    A = Os[y0:y0 + N + 1, x0:x0 + N + 1].astype(np.complex128)
    dy = (1.0 - fx) * (A[1:, :-1] - A[:-1, :-1]) + fx * (A[1:, 1:] - A[:-1, 1:])
    dx = (1.0 - fy) * (A[:-1, 1:] - A[:-1, :-1]) + fy * (A[1:, 1:] - A[1:, :-1])
    return dy, dx


# Fourier-shift variant of the sub-pixel patch: the N x N window at the integer corner,
# shifted by the fraction (fy, fx) with the shift theorem (periodic within the window).

def shift_phase(N: int, fy: float, fx: float) -> np.ndarray:
    """exp(2 pi i (ky fy + kx fx) / N) on the unshifted grid, k the signed frequency index."""
    k = np.fft.fftfreq(N) * N
    return np.exp(2j * math.pi * (k[:, None] * fy + k[None, :] * fx) / N)


def fourier_patch(Os: np.ndarray, y0: int, x0: int, fy: float, fx: float, N: int) -> np.ndarray:
    """Patch o(y, x) = O(y0 + fy + y, x0 + fx + x) by the shift theorem on the window."""
    w = Os[y0:y0 + N, x0:x0 + N].astype(np.complex128)
    return ifft2u(fft2u(w) * shift_phase(N, fy, fx))


def fourier_scatter(gOs: np.ndarray, g: np.ndarray, y0: int, x0: int, fy: float, fx: float) -> None:
    """Transpose of ``fourier_patch``: add the window gradient back into the slice."""
    N = g.shape[-1]
    gOs[y0:y0 + N, x0:x0 + N] += ifft2u(fft2u(g) * np.conj(shift_phase(N, fy, fx)))


def fourier_derivatives(Os: np.ndarray, y0: int, x0: int, fy: float, fx: float, N: int):
    """d(patch)/dy and d(patch)/dx of the Fourier-shifted patch (spectral derivative)."""
    k = np.fft.fftfreq(N) * N
    X = fft2u(Os[y0:y0 + N, x0:x0 + N].astype(np.complex128)) * shift_phase(N, fy, fx)
    dy = ifft2u(X * (2j * math.pi * k[:, None] / N))
    dx = ifft2u(X * (2j * math.pi * k[None, :] / N))
    return dy, dx


def probe_for_position(U: np.ndarray, w_k: Optional[np.ndarray]) -> np.ndarray:
    """Scan-point probe modes [M, N, N]: the weighted sum of the eigenprobes."""
    if w_k is None:
        return U[0].astype(np.complex128)
    return np.tensordot(w_k.astype(np.float64), U.astype(np.complex128), axes=(0, 0))


# ----------------------------------------------------------------------------- loss

def loss_and_factor(I: np.ndarray, Im: np.ndarray, loss: str, eps: float):
    """Per-pixel loss and dl/dI for the amplitude (Eq. (1)) or Poisson loss."""
    if loss == "amplitude":
        l = (np.sqrt(I) - np.sqrt(Im)) ** 2
        c = 1.0 - np.sqrt(Im / np.maximum(I, AMP_FLOOR))
    elif loss == "poisson":
        l = I - Im * np.log(I + eps)
        c = 1.0 - Im / (I + eps)
    else:
        raise ValueError(f"unknown loss {loss!r}")
    return l, c


# ----------------------------------------------------------------------------- model

def _as_inputs(obj, probe, positions, weights):
    O = np.asarray(obj).astype(np.complex128)
    if O.ndim == 2:
        O = O[None]
    U = np.asarray(probe).astype(np.complex128)
    if U.ndim == 3:
        U = U[None]
    r = np.asarray(positions).astype(np.float64).reshape(-1, 2)
    w = None if weights is None else np.asarray(weights).astype(np.float64).reshape(r.shape[0], -1)
    if w is None and U.shape[0] != 1:
        raise ValueError("several eigenprobes need weights")
    if w is not None and w.shape[1] != U.shape[0]:
        raise ValueError("weights must have one column per eigenprobe")
    return O, U, r, w


def _forward_one(O, P, y0, x0, fy, fx, tf, subpixel="bilinear"):
    """Exit waves of one position. Returns (patches o_s, incident waves psi_s [M,N,N]
    per slice, far-field Psi [M,N,N])."""
    S, N = O.shape[0], P.shape[-1]
    ext = fourier_patch if subpixel == "fourier" else extract_patch
    patches = [ext(O[s], y0, x0, fy, fx, N) for s in range(S)]
    psis = []
    psi = P
    for s in range(S):
        psis.append(psi)
        chi = psi * patches[s][None]
        if s < S - 1:
            psi = propagate(chi, tf)
    Psi = fft2u(chi)
    return patches, psis, Psi


def apply_A(obj, probe, positions, weights=None, lambda_z: float = 0.0) -> np.ndarray:
    """Far-field waves Psi [K, M, N, N] (unshifted) of every position and mode."""
    O, U, r, w = _as_inputs(obj, probe, positions, weights)
    N = U.shape[-1]
    tf = fresnel_tf(N, lambda_z) if O.shape[0] > 1 else None
    out = np.empty((r.shape[0], U.shape[1], N, N), dtype=np.complex128)
    for k in range(r.shape[0]):
        y0, x0, fy, fx = split_position(r[k], N, O.shape[1], O.shape[2], False)
        P = probe_for_position(U, None if w is None else w[k])
        out[k] = _forward_one(O, P, y0, x0, fy, fx, tf)[2]
    return out


def _backward_one(O, U, w_k, P, patches, psis, gPsi, tf, y0, x0, fy, fx,
                  gO, gU, want_w: bool, subpixel="bilinear", q2=None):
    """Adjoint of one position given dL/dPsi (g convention) for every mode.
    Accumulates into gO, gU; returns (per-slice patch gradients, dL/dw_k, dL/d(lambda z)).

    q2 (fy^2 + fx^2 on the unshifted grid) asks for the slice-spacing gradient: psi_s =
    F^-1(H F chi_{s-1}) with H = exp(-i pi lz q2), so d psi_s / d lz = F^-1((-i pi q2) H F
    chi_{s-1}) and, F being unitary, dL/dlz = sum_{s>0} Re sum_f conj(F g_psi_s) (-i pi q2)
    H F chi_{s-1}, with g_psi_s the gradient of the incident wave of slice s."""
    S = O.shape[0]
    g = ifft2u(gPsi)                                # [M, N, N] gradient of the last exit wave
    g_patch = [None] * S
    g_lz = 0.0
    for s in range(S - 1, -1, -1):
        g_patch[s] = np.sum(np.conj(psis[s]) * g, axis=0)
        g_psi = np.conj(patches[s])[None] * g       # gradient of the incident wave psi_s
        if s > 0:
            if q2 is not None:
                Gs = fft2u(g_psi)
                HX = tf * fft2u(psis[s - 1] * patches[s - 1][None])
                g_lz += float(np.sum(np.real(np.conj(Gs) * (-1j * math.pi * q2) * HX)))
            g = propagate_adjoint(g_psi, tf)
        else:
            g = g_psi
    gP = g                                          # gradient of the scan-point probe modes
    if w_k is None:
        gU[0] += gP
    else:
        gU += w_k[:, None, None, None] * gP[None]
    gw = None
    if want_w:
        gw = np.array([float(np.sum(np.real(np.conj(gP) * U[e]))) for e in range(U.shape[0])])
    scat = fourier_scatter if subpixel == "fourier" else scatter_patch
    for s in range(S):
        scat(gO[s], g_patch[s], y0, x0, fy, fx)
    return g_patch, gw, g_lz


def apply_AH(Y, obj, probe, positions, weights=None, lambda_z: float = 0.0):
    """Adjoint of the maps O_s -> Psi (other slices and probe fixed) and U -> Psi
    (object fixed), applied to Y [K, M, N, N].  Returns (g_obj [S,H,W], g_probe [E,M,N,N])."""
    O, U, r, w = _as_inputs(obj, probe, positions, weights)
    Y = np.asarray(Y).astype(np.complex128)
    N = U.shape[-1]
    tf = fresnel_tf(N, lambda_z) if O.shape[0] > 1 else None
    gO = np.zeros_like(O)
    gU = np.zeros_like(U)
    for k in range(r.shape[0]):
        y0, x0, fy, fx = split_position(r[k], N, O.shape[1], O.shape[2], False)
        wk = None if w is None else w[k]
        P = probe_for_position(U, wk)
        patches, psis, _ = _forward_one(O, P, y0, x0, fy, fx, tf)
        _backward_one(O, U, wk, P, patches, psis, Y[k], tf, y0, x0, fy, fx, gO, gU, False)
    return gO, gU


def forward(obj, probe, positions, I_meas, *, weights=None, loss: str = "amplitude",
            eps: float = 1e-3, lambda_z: float = 0.0, norm_count: Optional[float] = None,
            det_lambda_z: Optional[float] = None, subpixel: str = "bilinear"):
    """Loss L and the predicted intensity I_pred [K, N, N] (DC-centred in the far field,
    natural pixel order in the near field)."""
    out = forward_adjoint(obj, probe, positions, I_meas, weights=weights, loss=loss, eps=eps,
                          lambda_z=lambda_z, norm_count=norm_count, grads=(), det_lambda_z=det_lambda_z,
                          subpixel=subpixel)
    return out["loss"], out["I_pred"]


def forward_adjoint(obj, probe, positions, I_meas, *, weights=None, loss: str = "amplitude",
                    eps: float = 1e-3, lambda_z: float = 0.0, norm_count: Optional[float] = None,
                    grads: Sequence[str] = ("obj", "probe"),
                    det_lambda_z: Optional[float] = None, subpixel: str = "bilinear") -> Dict[str, np.ndarray]:
    """Loss, predicted intensity and the requested gradients
    (any of "obj", "probe", "pos", "weights", and "lambda_z").

    "lambda_z" is the gradient with respect to the wavelength-distance product of the
    model's Fresnel propagator: the slice spacing lambda_z of a multislice model (S > 1,
    far field; the slice spacing is a refinable parameter of the automatic-differentiation
    reconstructor, Reconstructors) or det_lambda_z of the near-field detector (S = 1). A
    model with neither, or with both, has no single lambda_z to differentiate (ValueError).

    Near field (det_lambda_z given; the propagation variant of the forward model, Software
    design, Overview): the last exit wave chi is carried to the detector by Fresnel
    propagation, Psi = F^-1(H F chi) with H = exp(-i pi lz_det (fy^2 + fx^2)), instead of
    the far-field transform; the detector is in natural pixel order. "lambda_z" asks for
    dL/d(lz_det) = sum_k,m Re sum_f conj(F g_Psi) (-i pi (fy^2 + fx^2)) H F chi.

    subpixel="fourier": the patch is the N x N window at the integer corner shifted by
    the fraction with the shift theorem (``fourier_patch``) instead of bilinear
    interpolation; the window is never widened."""
    near = det_lambda_z is not None
    if subpixel not in ("bilinear", "fourier"):
        raise ValueError(f"unknown subpixel model {subpixel!r}")
    fourier = subpixel == "fourier"
    O, U, r, w = _as_inputs(obj, probe, positions, weights)
    Im_all = np.asarray(I_meas).astype(np.float64)
    K, N = r.shape[0], U.shape[-1]
    S, H, W = O.shape
    Kn = float(K if (norm_count is None or norm_count <= 0) else norm_count)
    scale = 1.0 / (Kn * N * N)
    tf = fresnel_tf(N, lambda_z) if S > 1 else None
    want_pos = "pos" in grads
    want_w = "weights" in grads
    want_lz = "lambda_z" in grads
    if want_lz and near and S > 1:
        raise ValueError("lambda_z is ambiguous with both slices and a near-field detector")
    if want_lz and not near and S == 1:
        raise ValueError("a single-slice far-field model has no lambda_z")
    slice_lz = want_lz and S > 1
    if slice_lz:
        fq = np.fft.fftfreq(N)
        q2_slices = fq[:, None] ** 2 + fq[None, :] ** 2
        g_lz = 0.0
    any_grad = len(grads) > 0
    if near:
        tf_det = fresnel_tf(N, float(det_lambda_z))
        f = np.fft.fftfreq(N)
        q2 = f[:, None] ** 2 + f[None, :] ** 2
        g_lz = 0.0
    gO = np.zeros_like(O)
    gU = np.zeros_like(U)
    gr = np.zeros((K, 2))
    gw = np.zeros((K, U.shape[0]))
    I_pred = np.empty((K, N, N))
    total = 0.0
    for k in range(K):
        y0, x0, fy, fx = split_position(r[k], N, H, W, want_pos and not fourier)
        if fourier and (y0 + N > H or x0 + N > W):
            raise ValueError(f"scan window at {tuple(r[k])} leaves the {H}x{W} object")
        wk = None if w is None else w[k]
        P = probe_for_position(U, wk)
        patches, psis, Psi = _forward_one(O, P, y0, x0, fy, fx, tf, subpixel)
        if near:
            X = Psi                                   # F chi of the last exit wave
            Psi = ifft2u(tf_det * X)                  # detector-plane wave
        I = np.sum(np.abs(Psi) ** 2, axis=0)          # unshifted incoherent sum
        Im = Im_all[k] if near else uncentre(Im_all[k])
        l, c = loss_and_factor(I, Im, loss, eps)
        total += float(np.sum(l))
        I_pred[k] = I if near else centre(I)
        if not any_grad:
            continue
        gPsi = (2.0 * scale) * c[None] * Psi
        if near:
            Gd = fft2u(gPsi)
            if want_lz:
                g_lz += float(np.sum(np.real(np.conj(Gd) * (-1j * math.pi * q2) * tf_det * X)))
            gPsi = np.conj(tf_det) * Gd               # far-field-domain gradient of chi
        g_patch, gwk, glz = _backward_one(O, U, wk, P, patches, psis, gPsi, tf, y0, x0, fy, fx,
                                          gO, gU, want_w, subpixel, q2_slices if slice_lz else None)
        if slice_lz:
            g_lz += glz
        if want_w:
            gw[k] = gwk
        if want_pos:
            for s in range(S):
                dy, dx = (fourier_derivatives if fourier else patch_derivatives)(O[s], y0, x0, fy, fx, N)
                gr[k, 0] += float(np.sum(np.real(np.conj(g_patch[s]) * dy)))
                gr[k, 1] += float(np.sum(np.real(np.conj(g_patch[s]) * dx)))
    out: Dict[str, np.ndarray] = {"loss": total * scale, "I_pred": I_pred}
    if "obj" in grads:
        out["g_obj"] = gO
    if "probe" in grads:
        out["g_probe"] = gU
    if want_pos:
        out["g_pos"] = gr
    if want_w:
        out["g_weights"] = gw
    if want_lz:
        out["g_lambda_z"] = g_lz
    return out


def eq2_patch_gradient(obj, probe, position, I_meas, K_norm: float) -> np.ndarray:
    """Eq. (2) as printed, for one position, one mode, one slice and the amplitude loss:
    -(1/(B H W)) conj(p) (psi' - psi), with psi' the magnitude-updated wave brought back
    to the exit plane.  (Used to pin the adjoint against the paper's own formula.)"""
    O, U, r, _ = _as_inputs(obj, probe, position, None)
    N = U.shape[-1]
    y0, x0, fy, fx = split_position(r[0], N, O.shape[1], O.shape[2], False)
    o = extract_patch(O[0], y0, x0, fy, fx, N)
    p = U[0, 0]
    psi = p * o
    Psi = fft2u(psi)
    Im = uncentre(np.asarray(I_meas, dtype=np.float64).reshape(N, N))
    Psi_upd = np.sqrt(Im) * Psi / np.maximum(np.abs(Psi), math.sqrt(AMP_FLOOR))
    psi_upd = ifft2u(Psi_upd)
    return -(1.0 / (K_norm * N * N)) * np.conj(p) * (psi_upd - psi)


def patch_gradients(obj, probe, positions, I_meas, *, weights=None, loss="amplitude", eps=1e-3,
                    lambda_z=0.0, norm_count=None) -> np.ndarray:
    """Per-position, per-slice patch gradients g_o [K, S, N, N] before the scatter."""
    O, U, r, w = _as_inputs(obj, probe, positions, weights)
    Im_all = np.asarray(I_meas).astype(np.float64)
    K, N = r.shape[0], U.shape[-1]
    S, H, W = O.shape
    Kn = float(K if (norm_count is None or norm_count <= 0) else norm_count)
    tf = fresnel_tf(N, lambda_z) if S > 1 else None
    out = np.zeros((K, S, N, N), dtype=np.complex128)
    for k in range(K):
        y0, x0, fy, fx = split_position(r[k], N, H, W, False)
        wk = None if w is None else w[k]
        P = probe_for_position(U, wk)
        patches, psis, Psi = _forward_one(O, P, y0, x0, fy, fx, tf)
        I = np.sum(np.abs(Psi) ** 2, axis=0)
        _, c = loss_and_factor(I, uncentre(Im_all[k]), loss, eps)
        gPsi = (2.0 / (Kn * N * N)) * c[None] * Psi
        gO = np.zeros_like(O)
        gU = np.zeros_like(U)
        g_patch, _, _ = _backward_one(O, U, wk, P, patches, psis, gPsi, tf, y0, x0, fy, fx, gO, gU, False)
        for s in range(S):
            out[k, s] = g_patch[s]
    return out


# ----------------------------------------------------------------------------- preconditioner and scaling

def illumination(probe, positions, H: int, W: int, *, weights=None) -> np.ndarray:
    """Illumination in the object frame [H, W]: for every position, the probe intensity
    summed over modes, sum_m |P_{k,m}|^2, put back into the object frame by the
    transpose of the bilinear patch extraction, summed over positions. This is the
    object preconditioner built by superimposing the illumination function in the
    object frame (Introduction; its cost is discussed under Performance benchmarking)."""
    U = np.asarray(probe, dtype=np.complex128)
    N = U.shape[-1]
    pos = np.asarray(positions, dtype=np.float64)
    out = np.zeros((H, W), dtype=np.float64)
    for k in range(pos.shape[0]):
        w_k = None if weights is None else np.asarray(weights[k], dtype=np.float64)
        P = probe_for_position(U, w_k)
        A = np.sum(P.real ** 2 + P.imag ** 2, axis=0)
        y0, x0, fy, fx = split_position(pos[k], N, H, W, False)
        scatter_patch(out, A, y0, x0, fy, fx)
    return out


def probe_power_max(probe, K: int, *, weights=None) -> float:
    """max over positions and pixels of sum_m |P_{k,m}|^2."""
    U = np.asarray(probe, dtype=np.complex128)
    best = 0.0
    for k in range(K if weights is not None else 1):
        w_k = None if weights is None else np.asarray(weights[k], dtype=np.float64)
        P = probe_for_position(U, w_k)
        best = max(best, float(np.max(np.sum(np.abs(P) ** 2, axis=0))))
    return best


def normalized_gradients(g_obj, g_probe, obj, probe, K: int, *, weights=None, norm_count=None):
    """Scale-normalised gradients (Reconstructors, after Eq. (2)): the object gradient
    times B H W / max |p|^2, with B H W = K_norm N^2 here and max |p|^2 the largest
    mode-summed probe intensity; the probe gradient, read the same way, times
    K_norm N^2 / max |O|^2. A zero maximum leaves a gradient unchanged."""
    N = np.asarray(probe).shape[-1]
    c = float(norm_count if norm_count else K) * N * N
    go = gp = None
    if g_obj is not None:
        pm = probe_power_max(probe, K, weights=weights)
        go = np.asarray(g_obj, dtype=np.complex128) * (c / pm if pm > 0 else 1.0)
    if g_probe is not None:
        om = float(np.max(np.abs(np.asarray(obj, dtype=np.complex128)) ** 2))
        gp = np.asarray(g_probe, dtype=np.complex128) * (c / om if om > 0 else 1.0)
    return go, gp


# ----------------------------------------------------------------------------- probe modes

def orthogonalize_modes(probe):
    """Probe-mode orthogonalisation (a shared parameter routine, Software design /
    Overview): eigen-decomposition of the Gram matrix of eigenprobe 0's modes,
    G_mn = <P_m, P_n> = V diag(l) V^H, new modes P'_j = sum_m V_mj P_m with the
    eigenvalues in decreasing order (ties by index), the same V applied to every
    eigenprobe, and each column of V phased so that its largest-magnitude entry (the
    first on ties) is real and positive. Returns (new probe [E, M, N, N], l [M])."""
    U = np.asarray(probe, dtype=np.complex128)
    E, M = U.shape[:2]
    X = U[0].reshape(M, -1)
    G = X.conj() @ X.T
    lam, V = np.linalg.eigh(G)
    order = sorted(range(M), key=lambda j: (-lam[j], j))
    lam = lam[order]
    V = V[:, order]
    for j in range(M):
        a = np.abs(V[:, j])
        m = int(np.argmax(a))
        V[:, j] *= np.conj(V[m, j]) / a[m]
    out = np.einsum("mj,emab->ejab", V, U)
    return out, lam
