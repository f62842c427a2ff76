"""CPU oracle for the ordered tile-low-rank Matern log-likelihood.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import anything here.  The
GPU library never calls, links or falls back to this package, and this package
imports nothing from the GPU library.

Everything is plain float64 NumPy/SciPy, written to be checked against the
paper by eye:

* ``ordering``   -- encoding of coordinates, Morton and Hilbert keys, sorting,
                    KD-tree ordering, seeded random ordering (Section 3).
* ``matern``     -- the univariate Matern covariance (Section 4.1, eq. for
                    C_M) and dense covariance assembly (eq. for Sigma_ij).
* ``likelihood`` -- dense Gaussian log-likelihood (Section 1, eq. loglik).
* ``tlr``        -- exact per-tile SVD ranks (Section 2 / Section 3 intro) and
                    the likelihood of the tile-truncated covariance.
* ``blocked``    -- the dense likelihood by blocked Cholesky, for n up to 90,000.
* ``tgh``        -- Tukey g-and-h random fields (Section 4.2.2): the transform,
                    its inverse and the change-of-variables likelihood.

Parity pins (see tests/test_oracle_*.py): closed forms and special cases of
K_nu, brute-force determinants at high precision, an exact Markov
factorisation of the one-dimensional exponential model, the Hilbert curve
orders printed in the paper's Hilbert figure, Table "memory" magnitudes, and
structural invariants (bijections, permutation invariance, scaling laws).
"""
from . import ordering, matern, likelihood, tlr, tgh  # noqa: F401
