"""FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never does, and the two share no code.

Parity status: every function here is pinned by tests that do not re-use its own
formulas (brute-force DFT, closed forms, finite differences, adjoint identities,
reductions to simpler cases); none is "parity unpinned".
"""
from .ptycho_ref import (  # noqa: F401
    apply_A,
    apply_AH,
    centre,
    dft2_bruteforce,
    eq2_patch_gradient,
    extract_patch,
    fft2u,
    forward,
    forward_adjoint,
    fourier_patch,
    fourier_scatter,
    shift_phase,
    fresnel_tf,
    ifft2u,
    illumination,
    loss_and_factor,
    normalized_gradients,
    orthogonalize_modes,
    patch_derivatives,
    patch_gradients,
    probe_for_position,
    probe_power_max,
    propagate,
    scatter_patch,
    split_position,
    uncentre,
)
