"""RandRAND (randomized range deflation) preconditioned solver for MI355X (gfx950).

The compute path is the HIP library ``librandrand.so`` (C ABI in
``include/randrand.h``); this package only marshals arguments to it.  Importing
a function that needs the library raises ImportError if it was not built —
there is no CPU fallback.
"""
from .binding import (  # noqa: F401
    BLOCK_MAX, OP_DENSE, OP_MATERN32, OP_RBF, PREC_FP32, PREC_FP64, PREC_MIXED, RR_EBREAKDOWN, RR_EDEVICE,
    RR_EINVAL, RR_ENOCONV, RR_ENOMEM, RR_ENOTSPD, RR_OK, Operator, Precond, RRError,
    apply_operator, apply_operator_block, build_precond, dense_operator, kernel_operator, kernel_to_dense, lib,
    random_matrix, sketch, theta_apply,
)

__all__ = [
    "lib", "Operator", "Precond", "RRError", "build_precond", "dense_operator", "kernel_operator",
    "kernel_to_dense", "apply_operator", "apply_operator_block", "random_matrix", "sketch",
    "theta_apply",
]
