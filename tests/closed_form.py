"""Closed-form spectra used as pins (test helper, not part of the oracle).

The 1D factor h^-2 tridiag(-1 - g, 2, -1 + g) is a tridiagonal Toeplitz
matrix with eigenvalues h^-2 (2 - 2 sqrt((1-g)(1+g)) cos(j pi / (N+1))),
j = 1..N (a textbook result; for |g| < 1 they are real).  The 2D/3D
operators are Kronecker sums of such factors, so their eigenvalues are sums
of one factor eigenvalue per axis.
"""
import itertools

import numpy as np


def factor_eigs(N: int, beta: float) -> np.ndarray:
    h = 1.0 / (N + 1)
    g = beta * h / 2.0
    j = np.arange(1, N + 1)
    return (2.0 - 2.0 * np.sqrt(complex(1.0 - g * g)).real * np.cos(j * np.pi / (N + 1))) / (h * h)


def convdiff_eigs(N: int, beta) -> np.ndarray:
    """All eigenvalues of the D-dimensional operator, unsorted."""
    parts = [factor_eigs(N, b) for b in beta]
    tot = parts[0]
    for p in parts[1:]:
        tot = (tot[:, None] + p[None, :]).ravel()
    return tot
