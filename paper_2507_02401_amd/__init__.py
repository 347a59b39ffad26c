"""MI355X (gfx950) wavelet Sobolev-embedding / Matern-prior operators.

The wavelet realisation of the adjoint Sobolev embedding of arXiv 2507.02401 (Sec. 4):
E_s^* X = W^{-1}(D (W X)) with W a periodic orthonormal Daubechies DWT and D the
per-level weights, as hand-written HIP kernels behind a C ABI (include/eswave.h); and its
Fourier realisation (Sec. 4, Implementation), ifft(B fft(X)), with hipFFT transforms; and the
non-periodic (symmetric-extension) transform of Sec. 4 with its book-keeping band lengths.
"""
from ._lib import (OP_ADJOINT, OP_APPLY, OP_COV, OP_SAMPLE, EswaveError, load)
from .ops import (RaggedPlan, apply_op, autotune, es_adjoint, es_apply, fft_cov_apply, hs_norm_sq, matern_cov_apply,
                  matern_depth, matern_parameters, matern_sample, matern_to_s, plain_op, sym_band_lengths,
                  sym_cov_apply, sym_cov_apply_transpose, workspace_bytes)
from . import autograd

__all__ = ["autotune", "OP_ADJOINT", "OP_APPLY", "OP_COV", "OP_SAMPLE", "EswaveError", "load", "RaggedPlan", "apply_op",
           "es_adjoint", "es_apply", "fft_cov_apply", "hs_norm_sq", "matern_cov_apply", "matern_depth", "matern_parameters",
           "matern_sample", "matern_to_s",
           "plain_op", "sym_band_lengths", "sym_cov_apply", "sym_cov_apply_transpose", "workspace_bytes", "autograd"]
