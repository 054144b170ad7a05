"""MI355X (gfx950) additive-kernel Fourier fast summation for Gaussian processes.

Implements the hot path of "Preconditioned Additive Gaussian Processes with
Fourier Acceleration": NFFT-based products of additive Gaussian, Matern-1/2
and Matern-3/2 (and multiquadric, inverse multiquadric and sinc) kernel
matrices on feature windows of dimension <= 3 and of their hyper-parameter
derivatives, batched CG with FP64 scalars, the AAFN preconditioner and
preconditioned CG, stochastic Lanczos quadrature and the log-marginal-
likelihood gradient.  The numerical work runs
in hand-written HIP kernels behind the C ABI declared in include/nfftgp.h.
"""
from .plan import (AdditiveKernelPlan, GAUSS, MATERN12, MATERN32, MQ, IMQ, SINC, SCALE_AUTO, SCALE_NONE,  # noqa: F401
                   slq_logquad)
from .gp import khat_apply, lml_estimate, lml_surrogate  # noqa: F401
from .model import AdditiveGP  # noqa: F401
from ._lib import NfftgpError, LIB_PATH  # noqa: F401
