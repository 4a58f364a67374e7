"""Seeded synthetic ptychography workloads (configs 0-5) and noise draws.

Everything here is input preparation: smooth random objects, probe shapes,
scan geometries, the perturbation that moves a problem off its truth, and
Poisson photon counting. No propagation, patch extraction or loss is computed
here; the caller forms clean intensities with whichever forward model it tests.

Positions are float32 (y, x): the top-left corner of the N x N frame in object
pixels. The integer part is the floor, the rest is the sub-pixel fraction.

Seeds: numpy.random.default_rng(20929 + config) for the truth, and the seed
given to ``perturb`` / ``poisson_counts`` for the rest.  The order of draws in
each builder is fixed by the code below (top to bottom).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import List, Optional, Tuple

import numpy as np
from numpy.polynomial.hermite import hermval
from scipy.ndimage import gaussian_filter

SEED_BASE = 20929
PHOTONS_PER_FRAME = 1.0e4


@dataclass
class Problem:
    """One forward/adjoint problem instance (all arrays host, float32/complex64)."""

    name: str
    obj: np.ndarray                 # complex64 [S, H, W]
    probe: np.ndarray               # complex64 [E, M, N, N]
    positions: np.ndarray           # float32 [K, 2]  (y, x) frame top-left
    weights: Optional[np.ndarray]   # float32 [K, E] or None (then E == 1, w == 1)
    loss: str                       # "amplitude" | "poisson"
    eps: float = 1.0e-3             # Poisson regulariser, photons
    lambda_z: float = 0.0           # slice-to-slice Fresnel product, px^2
    grads: Tuple[str, ...] = ("obj", "probe")
    det_lambda_z: Optional[float] = None  # near-field detector (Fresnel), or None: far field
    subpixel: str = "bilinear"            # sub-pixel patch model: "bilinear" or "fourier"

    @property
    def N(self) -> int:
        return int(self.probe.shape[-1])

    @property
    def M(self) -> int:
        return int(self.probe.shape[1])

    @property
    def E(self) -> int:
        return int(self.probe.shape[0])

    @property
    def S(self) -> int:
        return int(self.obj.shape[0])

    @property
    def K(self) -> int:
        return int(self.positions.shape[0])

    @property
    def H(self) -> int:
        return int(self.obj.shape[1])

    @property
    def W(self) -> int:
        return int(self.obj.shape[2])

    def subset(self, idx) -> "Problem":
        """The same problem restricted to the scan points ``idx``."""
        idx = np.asarray(idx)
        w = None if self.weights is None else np.ascontiguousarray(self.weights[idx])
        return replace(self, positions=np.ascontiguousarray(self.positions[idx]), weights=w)


# ----------------------------------------------------------------------------- fields

def smooth_field(shape, sigma: float, rng: np.random.Generator, dist: str = "normal") -> np.ndarray:
    """White noise smoothed by a periodic Gaussian (sigma px) over the last two axes,
    rescaled to zero mean and unit standard deviation."""
    if dist == "uniform":
        x = rng.uniform(0.0, 1.0, size=shape)
    else:
        x = rng.standard_normal(size=shape)
    sig = [0.0] * (len(shape) - 2) + [sigma, sigma]
    x = gaussian_filter(x, sigma=sig, mode="wrap")
    x = x - x.mean()
    return x / max(float(x.std()), 1e-30)


def _rescale(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    mn, mx = float(x.min()), float(x.max())
    return lo + (hi - lo) * (x - mn) / max(mx - mn, 1e-30)


def random_object(rng, H: int, W: int, amp=(0.8, 1.0), phase=(-0.5, 0.5), sigma: float = 2.0) -> np.ndarray:
    """Amplitude and phase drawn uniform, smoothed (sigma px) and mapped back onto the
    stated ranges; returns complex64 [H, W]."""
    a = _rescale(smooth_field((H, W), sigma, rng, "uniform"), *amp)
    p = _rescale(smooth_field((H, W), sigma, rng, "uniform"), *phase)
    return (a * np.exp(1j * p)).astype(np.complex64)


def _centred_grid(N: int):
    c = (N - 1) / 2.0
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    return y - c, x - c


def disk_probe(N: int, radius: float, sigma: float = 2.0) -> np.ndarray:
    """Gaussian-apodised disk with quadratic phase pi r^2 / R^2 (complex128 [N, N])."""
    y, x = _centred_grid(N)
    r2 = y * y + x * x
    disk = (r2 <= radius * radius).astype(np.float64)
    amp = gaussian_filter(disk, sigma=sigma, mode="constant")
    return amp * np.exp(1j * math.pi * r2 / (radius * radius))


def hermite_gauss(N: int, m: int, n: int, w0: float) -> np.ndarray:
    """Hermite-Gaussian HG(m, n) with waist w0 px (real [N, N]); m along x, n along y."""
    y, x = _centred_grid(N)
    cm = np.zeros(m + 1)
    cm[m] = 1.0
    cn = np.zeros(n + 1)
    cn[n] = 1.0
    s = math.sqrt(2.0) / w0
    return hermval(s * x, cm) * hermval(s * y, cn) * np.exp(-(x * x + y * y) / (w0 * w0))


def orthonormalise(modes: np.ndarray) -> np.ndarray:
    """QR-orthonormalise a stack of complex fields [M, N, N] (unit norm each)."""
    M = modes.shape[0]
    A = modes.reshape(M, -1).T
    q, r = np.linalg.qr(A)
    # keep the sign/phase of the original leading coefficients
    d = np.diag(r)
    ph = d / np.maximum(np.abs(d), 1e-300)
    q = q * ph[None, :]
    return q.T.reshape(modes.shape)


def _photon_scale(probe0: np.ndarray, obj: np.ndarray, photons: float) -> float:
    """Factor for the probe so that (sum of mode powers) x mean |O|^2 = photons."""
    power = float(np.sum(np.abs(probe0) ** 2))
    mean_t = float(np.mean(np.abs(obj.astype(np.complex128)) ** 2))
    return math.sqrt(photons / max(power * mean_t, 1e-300))


# ----------------------------------------------------------------------------- scans

def raster(ny: int, nx: int, step: float, start_y: float = 0.0, start_x: float = 0.0) -> np.ndarray:
    iy, ix = np.mgrid[0:ny, 0:nx]
    pos = np.stack([start_y + step * iy.ravel(), start_x + step * ix.ravel()], axis=1)
    return pos.astype(np.float64)


def fermat_spiral(K: int, cy: float, cx: float, rmax: float) -> np.ndarray:
    n = np.arange(K, dtype=np.float64)
    r = rmax * np.sqrt(n / max(K - 1, 1))
    th = np.deg2rad(137.508) * n
    return np.stack([cy + r * np.sin(th), cx + r * np.cos(th)], axis=1)


# ----------------------------------------------------------------------------- configs

def _config0(rng, H: int, K: Optional[int]) -> Problem:
    N = 64
    obj = random_object(rng, H, H)[None]
    probe = disk_probe(N, 20.0, 2.0)[None, None]
    side = (H - N) // 8 + 1
    pos = raster(side, side, 8.0)
    if K is not None:
        pos = pos[:K]
    probe = probe * _photon_scale(probe[0], obj, PHOTONS_PER_FRAME)
    return Problem("c0", obj, probe.astype(np.complex64), pos.astype(np.float32), None,
                   "amplitude", grads=("obj", "probe"))


def _hg_modes(N: int, orders, w0: float, powers, curvature_radius: float) -> np.ndarray:
    y, x = _centred_grid(N)
    qphase = np.exp(1j * math.pi * (x * x + y * y) / (curvature_radius ** 2))
    modes = np.stack([hermite_gauss(N, m, n, w0) * qphase for (m, n) in orders]).astype(np.complex128)
    modes = orthonormalise(modes)
    return modes * np.sqrt(np.asarray(powers, dtype=np.float64))[:, None, None]


def _config1(rng, H: int, K: int) -> Problem:
    N = 128
    obj = random_object(rng, H, H)[None]
    modes = _hg_modes(N, [(0, 0), (1, 0), (0, 1), (1, 1)], 16.0, [0.7, 0.15, 0.1, 0.05], 32.0)
    centre = float((H - N - 2) // 2)
    pos = fermat_spiral(K, centre, centre, centre - 1.0)
    pos = np.floor(pos) + rng.uniform(0.0, 1.0, size=pos.shape)
    probe = modes[None] * _photon_scale(modes, obj, PHOTONS_PER_FRAME)
    return Problem("c1", obj, probe.astype(np.complex64), pos.astype(np.float32), None,
                   "poisson", eps=1e-3, grads=("obj", "probe", "pos"))


def _config2(rng, H: int, K: int) -> Problem:
    N = 256
    obj = random_object(rng, H, H)[None]
    radius = 14.0
    u0 = disk_probe(N, radius, 2.0)
    env = np.abs(u0)
    y, x = _centred_grid(N)
    orders = [(1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (0, 3)]
    s = math.sqrt(2.0) / radius
    eig = [u0]
    for (m, n) in orders:
        cm = np.zeros(m + 1)
        cm[m] = 1.0
        cn = np.zeros(n + 1)
        cn[n] = 1.0
        eig.append(hermval(s * x, cm) * hermval(s * y, cn) * env * np.exp(1j * np.angle(u0)))
    U = orthonormalise(np.stack(eig).astype(np.complex128))
    side = int(math.ceil(math.sqrt(K)))
    step = 17.0
    start = math.floor((H - N - 1 - (side - 1) * step) / 2.0)
    if start < 2:
        raise ValueError("object too small for the jittered raster")
    pos = raster(side, side, step, start, start)[:K]
    pos = pos + rng.uniform(-2.0, 2.0, size=pos.shape)
    w = np.empty((K, 8), dtype=np.float64)
    w[:, 0] = rng.normal(1.0, 0.1, size=K)
    w[:, 1:] = rng.normal(0.0, 0.05, size=(K, 7))
    U = U * _photon_scale(U[0:1], obj, PHOTONS_PER_FRAME)
    return Problem("c2", obj, U[:, None].astype(np.complex64), pos.astype(np.float32),
                   w.astype(np.float32), "amplitude", grads=("obj", "probe", "weights"))


def fresnel_number_lambda_z(N: int, nf: float = 50.0) -> float:
    """lambda*z in px^2 for Fresnel number nf with N_F = (N/2)^2 / (lambda z)."""
    return (N / 2.0) ** 2 / nf


def _config3(rng, S: int, H: int, K: int) -> Problem:
    N = 128
    ph = np.stack([_rescale(smooth_field((H, H), 2.0, rng, "uniform"), 0.0, 0.1) for _ in range(S)])
    obj = np.exp(1j * ph).astype(np.complex64)
    modes = _hg_modes(N, [(0, 0), (1, 0)], 16.0, [0.8, 0.2], 32.0)
    centre = (H - N - 1) / 2.0
    pos = fermat_spiral(K, centre, centre, centre - 1.5)
    probe = modes[None] * _photon_scale(modes, obj[0], PHOTONS_PER_FRAME)
    return Problem("c3", obj, probe.astype(np.complex64), pos.astype(np.float32), None,
                   "amplitude", lambda_z=fresnel_number_lambda_z(N), grads=("obj", "probe", "pos"))


def _mode_orders(M: int):
    """The first M Hermite-Gauss orders (m, n), by total order m + n, then by m."""
    orders = []
    tot = 0
    while len(orders) < M:
        for m in range(tot, -1, -1):
            orders.append((m, tot - m))
        tot += 1
    return orders[:M]


def _config5(rng, H: int, W: int, K: int, M: int) -> Problem:
    """Mode-heavy workload shaped like the paper's benchmark dataset: 6732 diffraction
    patterns of 128^2, a 413 x 535 object and 30 probe modes (no OPR). The probe modes
    are orthonormalised Hermite-Gauss modes with powers decaying as exp(-j / 6); the scan
    is a 68 x 99 raster covering the object (step about 4.1 px) with sub-pixel offsets."""
    N = 128
    obj = random_object(rng, H, W)[None]
    powers = np.exp(-np.arange(M) / 6.0)
    powers = powers / powers.sum()
    modes = _hg_modes(N, _mode_orders(M), 16.0, powers, 32.0)
    ny, nx = 68, 99
    step = min((H - N - 2) / (ny - 1), (W - N - 2) / (nx - 1))
    pos = raster(ny, nx, step) + rng.uniform(0.0, 1.0, size=(ny * nx, 2))
    pos = pos[:K]
    probe = modes[None] * _photon_scale(modes, obj, PHOTONS_PER_FRAME)
    return Problem("c5", obj, probe.astype(np.complex64), pos.astype(np.float32), None,
                   "amplitude", grads=("obj", "probe", "pos"))


def _config6(rng, N: int, K: int) -> Problem:
    """The supplement's speed-benchmark shape: 961 diffraction patterns, 15 incoherent probe
    modes and 3 OPR eigenprobes (the primary one included), frames of 128^2 or 512^2,
    amplitude loss, position correction disabled (object, eigenprobe and weight gradients).
    The paper states no object, scan or probe for it: a 31 x 31 raster at N / 16 px steps
    with sub-pixel offsets over an object of scan extent + N + 4; eigenprobe 0 holds 15
    orthonormal Hermite-Gauss modes (waist N / 8, powers exp(-j / 4)); eigenprobes 1 and 2
    are the same modes times smooth random fields (the slow drift OPR models); weights
    N(1, 0.1) for the primary eigenprobe and N(0, 0.05) for the others."""
    M, E = 15, 3
    side = 31
    step = N / 16.0
    H = int(math.ceil((side - 1) * step)) + N + 4
    obj = random_object(rng, H, H)[None]
    powers = np.exp(-np.arange(M) / 4.0)
    powers = powers / powers.sum()
    modes = _hg_modes(N, _mode_orders(M), N / 8.0, powers, N / 4.0)
    eig = [modes]
    for _ in range(E - 1):
        field = smooth_field((N, N), N / 16.0, rng) + 1j * smooth_field((N, N), N / 16.0, rng)
        eig.append(modes * (0.5 * field)[None])
    U = np.stack(eig)
    pos = raster(side, side, step, 1.0, 1.0) + rng.uniform(0.0, 1.0, size=(side * side, 2))
    pos = pos[:K]
    w = np.empty((pos.shape[0], E), dtype=np.float64)
    w[:, 0] = rng.normal(1.0, 0.1, size=pos.shape[0])
    w[:, 1:] = rng.normal(0.0, 0.05, size=(pos.shape[0], E - 1))
    U = U * _photon_scale(U[0], obj, PHOTONS_PER_FRAME)
    return Problem(f"c6n{N}", obj, U.astype(np.complex64), pos.astype(np.float32), w.astype(np.float32),
                   "amplitude", grads=("obj", "probe", "weights"))


def make_config(c: int, *, H: Optional[int] = None, K: Optional[int] = None,
                S: Optional[int] = None, W: Optional[int] = None, M: Optional[int] = None,
                N: Optional[int] = None) -> Problem:
    """Truth problem for config ``c`` (0-3, 5, 6). H, K, S shrink it for tests while keeping
    the frame size, the mode/eigenprobe structure and the scan pattern (config 5 also
    takes W and the mode count M; config 6 takes the frame size N, 128 or 512, and K)."""
    rng = np.random.default_rng(SEED_BASE + c)
    if c == 0:
        return _config0(rng, H or 256, K)
    if c == 1:
        return _config1(rng, H or 1024, K or 2000)
    if c == 2:
        return _config2(rng, H or 2048, K or 10000)
    if c == 3:
        return _config3(rng, S or 8, H or 2048, K or 5000)
    if c == 5:
        return _config5(rng, H or 413, W or 535, K or 6732, M or 30)
    if c == 6:
        return _config6(rng, N or 128, K or 961)
    raise ValueError(f"unknown config {c}")


def make_batched_config(n_datasets: int = 32, *, sizes=(64, 128, 256, 512), k_range=(200, 5000),
                        max_modes: int = 4, seed: int = SEED_BASE + 4, k_scale: float = 1.0) -> List[Problem]:
    """Config 4: independent datasets of uneven frame size. Each has a raster scan at
    step 0.4 N (probe diameter about N/2, about 20% linear overlap), sub-pixel offsets,
    a per-position probe amplitude w_k ~ U[0.85, 1.15] applied to every mode (E = 1),
    and an object sized to the scan extent plus the frame. ``k_scale`` shrinks K."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_datasets):
        N = int(rng.choice(np.asarray(sizes)))
        M = int(rng.integers(1, max_modes + 1))
        K = int(round(math.exp(rng.uniform(math.log(k_range[0]), math.log(k_range[1])))))
        K = max(1, int(round(K * k_scale)))
        side = int(math.ceil(math.sqrt(K)))
        step = 0.4 * N
        Hs = int(math.ceil((side - 1) * step)) + N + 2
        obj = random_object(rng, Hs, Hs)[None]
        orders = [(0, 0), (1, 0), (0, 1), (1, 1)][:M]
        powers = np.asarray([0.7, 0.15, 0.1, 0.05][:M])
        powers = powers / powers.sum()
        modes = _hg_modes(N, orders, N / 8.0, powers, N / 4.0)
        pos = raster(side, side, step)[:K] + rng.uniform(0.0, 1.0, size=(K, 2))
        w = rng.uniform(0.85, 1.15, size=(K, 1))
        probe = modes[None] * _photon_scale(modes, obj, PHOTONS_PER_FRAME)
        out.append(Problem(f"c4.{i}", obj, probe.astype(np.complex64), pos.astype(np.float32),
                           w.astype(np.float32), "amplitude", grads=("obj", "probe", "pos", "weights")))
    return out


# ----------------------------------------------------------------------------- perturbation, noise

def perturb(p: Problem, seed: int, obj_amp: float = 0.1, probe_amp: float = 0.05,
            pos_amp: float = 0.5, weight_amp: float = 0.02) -> Problem:
    """A start point off the truth: O * exp(0.1 (n1 + i n2)), P + 5% smoothed noise,
    r + U[-0.5, 0.5] px (kept inside the object with a one-pixel margin), w + N(0, 0.02)."""
    rng = np.random.default_rng(seed)
    n1 = smooth_field(p.obj.shape, 2.0, rng)
    n2 = smooth_field(p.obj.shape, 2.0, rng)
    obj = (p.obj.astype(np.complex128) * np.exp(obj_amp * (n1 + 1j * n2))).astype(np.complex64)
    pr = p.probe.astype(np.complex128)
    scale = float(np.abs(pr).max())
    m1 = smooth_field(pr.shape, 2.0, rng)
    m2 = smooth_field(pr.shape, 2.0, rng)
    probe = (pr + probe_amp * scale * (m1 + 1j * m2)).astype(np.complex64)
    pos = p.positions.astype(np.float64) + rng.uniform(-pos_amp, pos_amp, size=p.positions.shape)
    hi_y = p.H - p.N - 1.0 - 1e-3
    hi_x = p.W - p.N - 1.0 - 1e-3
    pos[:, 0] = np.clip(pos[:, 0], 0.0, hi_y)
    pos[:, 1] = np.clip(pos[:, 1], 0.0, hi_x)
    w = None
    if p.weights is not None:
        w = (p.weights.astype(np.float64) + rng.normal(0.0, weight_amp, size=p.weights.shape)).astype(np.float32)
    return replace(p, obj=obj, probe=probe, positions=pos.astype(np.float32), weights=w)


def poisson_counts(I_clean: np.ndarray, seed: int) -> np.ndarray:
    """Photon counts ~ Poisson(I_clean), float32."""
    rng = np.random.default_rng(seed)
    lam = np.maximum(np.asarray(I_clean, dtype=np.float64), 0.0)
    return rng.poisson(lam).astype(np.float32)
