"""ptyhip: MI355X-native forward model and adjoint of gradient-based ptychography
(arxiv 2510.20929). The compute path is the HIP library libptyhip.so behind the C ABI
of include/ptyhip.h; this package binds it (ctypes) and adds the autograd and batched
forms. Importing the package does not load the library; the first call does, and
fails loudly if it has not been built.
"""
from .ptyhip import (  # noqa: F401
    ACCUMULATE, BATCH_PER_CALL, Batch, FLAG_BOUNDS, FLAG_NONFINITE, GRAD_OBJ, GRAD_POS, GRAD_PROBE, GRAD_WEIGHTS, LOSS_AMPLITUDE,
    LOSS_POISSON, PLAIN, Desc, Plan, PtyhipError, lib, make_desc, ptyhip_desc_validate,
)

from .autograd import PtychoLoss, ptycho_loss  # noqa: F401,E402

__all__ = ["Plan", "PtyhipError", "PtychoLoss", "make_desc", "ptycho_loss", "ptyhip_desc_validate", "lib"]
