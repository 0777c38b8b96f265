"""The named benchmark workloads and their solver parameters.

Each entry gives the operator recipe and the rKS parameters (k wanted pairs,
Krylov dimension m, sketch size d, which part of the spectrum, tolerance, sketch
kind / seed, start seed, basis precision).  Sketch seeds and kinds the workload
description leaves open are fixed here: sparse-sign with 8 nonzeros per column
(the paper's setting, Section 5) and seed equal to the workload's index.
"""
import numpy as np

from .convdiff import convdiff2d, convdiff3d, convdiff2d_field
from .randsparse import powerlaw_random
from .tridiag import tridiag_noisy

CONFIGS = {
    # 2D convection-diffusion, 100^2, closed-form spectrum, Gaussian sketch.
    "cd2d-100": dict(matrix=lambda: convdiff2d(100, (20.0, 10.0)), k=10, m=40, d=80,
                     which="LR", tol=1e-10, sketch="gauss", zeta=8, sketch_seed=0,
                     start_seed=1, lock=True, precision="fp64"),
    # Same operator on 1000^2, smallest real part, with locking.
    "cd2d-1000": dict(matrix=lambda: convdiff2d(1000, (50.0, 30.0)), k=20, m=60, d=240,
                      which="SR", tol=1e-10, sketch="sparse", zeta=8, sketch_seed=2,
                      start_seed=1, lock=True, precision="fp64"),
    # 3D convection-diffusion 160^3, largest real part, low-precision basis.
    "cd3d-160": dict(matrix=lambda: convdiff3d(160, (40.0, 20.0, 10.0)), k=30, m=90, d=360,
                     which="LR", tol=1e-10, sketch="sparse", zeta=8, sketch_seed=3,
                     start_seed=1, lock=True, precision="fp32"),
    # Random power-law sparse matrix, largest modulus.
    "powerlaw-2m": dict(matrix=lambda: powerlaw_random(2_000_000, 4), k=50, m=120, d=480,
                        which="LM", tol=1e-10, sketch="sparse", zeta=8, sketch_seed=4,
                        start_seed=1, lock=True, precision="fp64"),
    # Parametric 2D family on 512^2 (instance 0 shown; instance i uses seed 10000+i).
    "cd2d-512-field": dict(matrix=lambda: convdiff2d_field(512, 10000), k=16, m=48, d=192,
                           which="SR", tol=1e-10, sketch="sparse", zeta=8, sketch_seed=5,
                           start_seed=1, lock=True, precision="fp64"),
    # The paper's synthetic tridiagonal family (Section 5.1): k = 40, m = 2k,
    # sparse-sign sketch with d = 2m; exponential spectrum at its largest n.
    "tridiag-exp-5m-lm": dict(matrix=lambda: tridiag_noisy(5_000_000, "exponential", 7), k=40, m=80, d=160,
                              which="LM", tol=1e-10, sketch="sparse", zeta=8, sketch_seed=7,
                              start_seed=1, lock=True, precision="fp64"),
    # Same matrix, smallest modulus, a fixed 10 restarts (no convergence expected).
    "tridiag-exp-5m-sm10": dict(matrix=lambda: tridiag_noisy(5_000_000, "exponential", 7), k=40, m=80, d=160,
                                which="SM", tol=1e-10, sketch="sparse", zeta=8, sketch_seed=7,
                                start_seed=1, lock=True, precision="fp64", max_restarts=10),
}


def named_config(name: str) -> dict:
    """Return a copy of the parameters of workload ``name`` (matrix not built)."""
    cfg = dict(CONFIGS[name])
    cfg["name"] = name
    return cfg


def start_vector_normal(n: int, seed: int) -> np.ndarray:
    """An i.i.d. N(0,1) test vector drawn with NumPy's PCG64 (a plain input
    for kernel tests; the solver's own seeded start uses its counter-based
    generator instead)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)
