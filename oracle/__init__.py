"""Plain FP64 CPU oracle for randomized Krylov-Schur (rKS).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library may import, call or link
anything here; only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the GPU path: its random embedding is built
from its own implementation of the written Philox4x32-10 counter-based
generator, and its small dense linear algebra is LAPACK through SciPy.

Modules:
  philox  -- Philox4x32-10 (Salmon et al., SC'11), uniforms, Box-Muller.
  sketch  -- the random embedding Omega (Gaussian or sparse-sign), explicit.
  rks     -- Algorithms 1 and 2 of the paper with residual monitoring
             (Section 4.1), locking (Sections 4.2-4.4) and whitening
             (Section 3.3), step by step in the paper's order.
  convnet -- the learned-start network (dilated 3x3 convolutions, subspace
             loss, Adam, bilinear resampling) written out with loops.

Parity status: every function is pinned by a test under tests/ (known-answer
vectors, closed-form spectra, dense brute force, exact identities of the
decomposition); see the header of each module.
"""
from .philox import philox4x32_10, uniform01, box_muller, start_vector
from .sketch import sketch_matrix, sparse_sign_columns
from .rks import RKSOracle, rks, eigpairs, which_key

__all__ = ["philox4x32_10", "uniform01", "box_muller", "start_vector", "sketch_matrix",
           "sparse_sign_columns", "RKSOracle", "rks", "eigpairs", "which_key"]
