"""FP64 CPU oracle for hierarchical-matrix maximum likelihood (Chen & Anitescu).

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct NumPy/SciPy code that
states what the method computes.  Only the test suite, the package smoke check
and the CPU-baseline leg of the benchmark may import it; the HIP library never
does, and this package imports nothing from the HIP library.

Modules
  model     -- the stencil operators, dense K(theta) and dK/dtheta assembled from
               K-applied-to-unit-vectors (Sec. 2.1), and the KD-tree ordering (Sec. 5.2).
  exact     -- log-likelihood, score and Fisher information from their definitions
               (Sec. 2.2, eqs. "log-like", "score", "fisher info") on any dense SPD K.
  spectral  -- closed form of the same quantities via the sine-transform
               eigenbasis of the Dirichlet stencils (independent of `model`).
  peeling   -- dense replay of the randomized peeling construction (Sec. 3.2,
               Alg. 1) and of its derivative (Sec. 3.3, Alg. 2), giving K~ and K~_j.
  mle       -- maximum-likelihood fits by Fisher scoring on the exact likelihood
               (dense or closed form; Sec. 2, eqs. "score", "fisher info", "CLT").

Every function cites the passage it follows.  Parity status is listed per
module; every function here is pinned by a test in tests/test_oracle_*.py.
"""
