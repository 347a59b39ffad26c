"""FP64 CPU oracle for the wavelet Sobolev-embedding / Matern-prior operators.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link this package; only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
code, tables or constants with the GPU path: the Daubechies filters are
derived here independently (mpmath spectral factorisation) and the transforms
are written as plain modular-index gathers over whole arrays, in float64.

Paper: Kultima, Ramlau, Sahlstrom, Tarvainen, "Fast reconstruction approaches
for photoacoustic tomography with smoothing Sobolev/Matern priors"
(arXiv 2507.02401).  The operator realised here is the wavelet form of the
adjoint Sobolev embedding, Sec. 4 (Prop. 4.2, the level-weight rule and the
block-diagonal matrix D, and the formula E_s^* X = W^{-1}(D (W X))).

Pinning status (see tests/test_oracle_*.py):
  * filters      -- pinned by the orthonormality / vanishing-moment /
                    minimum-phase invariants (which determine dbN uniquely),
                    the db2 closed form and the Haar filter;
  * transforms   -- pinned by perfect reconstruction, Parseval, dense
                    Kronecker brute force, vanishing moments;
  * level weights and alignment -- pinned by the Haar block-mean closed form
                    and the spectrum closed form;
  * operators    -- pinned by the identities s=0 / m=0, constants preserved,
                    brute-force adjointness, the semigroup and square-root
                    identities;
  * Tikhonov solve -- pinned by a dense direct solve of the normal equations
                    on tiny grids and by the first-order optimality condition;
  * Fourier form of E_s^* (Sec. 4, Implementation) -- pinned by plane-wave eigenvalues (closed
                    form, aliased wave numbers included), a point-by-point DFT
                    sum on tiny grids and its invariants (identity at s = 0,
                    semigroup, symmetry, shift equivariance).
  * symmetric-extension transform and W^{-1} D W (Sec. 4: MATLAB's transform,
                    band lengths in a book-keeping matrix) -- pinned by the periodic
                    transform of the mirrored signal (analysis) and of zero-padded
                    coefficients (synthesis), the Haar hand example, perfect
                    reconstruction, dense W^{-1} W = I, equality with the periodic
                    operator for Haar on dyadic sides, identities at s = 0 and for
                    constants, and the low-pass recurrence;
  The absolute Matern scale constant of Cor. 4.3 is not part of the path and
  is not implemented (parity unpinned; the constant is dropped as Remark 3.3
  allows).
"""

from .filters import daubechies_lowpass, quadrature_highpass
from .dwt import analysis_axis, synthesis_axis, dwt, idwt, level_weights, weight_map
from .ops import es_adjoint, es_apply, matern_cov_apply, matern_sample, hs_norm_sq
from .solver import tikhonov_gmres, tikhonov_solve
from .fourier import fft_cov_apply, fourier_multiplier
from .symdwt import sym_cov_apply, sym_dwt, sym_idwt, sym_lengths
from . import dense

__all__ = [
    "daubechies_lowpass", "quadrature_highpass",
    "analysis_axis", "synthesis_axis", "dwt", "idwt", "level_weights", "weight_map",
    "es_adjoint", "es_apply", "matern_cov_apply", "matern_sample", "hs_norm_sq",
    "tikhonov_solve", "tikhonov_gmres", "fft_cov_apply", "fourier_multiplier", "dense",
]
