"""Seeded synthetic input generators for the randomized Krylov-Schur eigensolver.

This package builds the sparse test operators (CSR arrays) and nothing else: it
holds none of the eigensolver's arithmetic, so that both the GPU library's
callers and the CPU oracle can draw the same inputs from it without sharing any
method code.

Operators:
  * ``convdiff2d`` / ``convdiff3d``: the 5- and 7-point central finite-difference
    discretisation of -Laplace(u) + beta . grad(u) on the unit square / cube
    with homogeneous Dirichlet conditions, unknowns numbered x-fastest.
  * ``convdiff2d_field``: the same 2D operator with a spatially varying
    velocity field beta(x, y) built from random Fourier modes.
  * ``powerlaw_random``: a random non-symmetric sparse matrix with power-law
    row lengths.
  * ``tridiag_noisy``: the synthetic tridiagonal family of the paper's first
    experiment (Section 5.1, Table "SynthTestMatrices").
  * ``named_config``: the five benchmark workloads by name.
"""
from .csr import CSR
from .convdiff import convdiff2d, convdiff3d, convdiff2d_field, fourier_beta_field
from .randsparse import powerlaw_random, powerlaw_exponent
from .tridiag import tridiag_noisy
from .configs import CONFIGS, named_config, start_vector_normal

__all__ = [
    "CSR", "convdiff2d", "convdiff3d", "convdiff2d_field", "fourier_beta_field",
    "powerlaw_random", "powerlaw_exponent", "tridiag_noisy", "CONFIGS",
    "named_config", "start_vector_normal",
]
