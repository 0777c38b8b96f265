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


def factor_kappa(N: int, beta: float) -> np.ndarray:
    """Eigenvalue condition numbers of the 1D factor (|g| < 1): right
    eigenvectors r^i sin(i j pi/(N+1)), left ones r^-i sin(i j pi/(N+1)),
    r = sqrt((1+g)/(1-g)); kappa_j = |v||w| / |w^T v| with w^T v = (N+1)/2."""
    h = 1.0 / (N + 1)
    g = beta * h / 2.0
    r = np.sqrt((1.0 + g) / (1.0 - g))
    i = np.arange(1, N + 1)
    kap = np.empty(N)
    for j in range(1, N + 1):
        s = np.sin(i * j * np.pi / (N + 1))
        v = r ** i * s
        w = r ** (-i) * s
        kap[j - 1] = np.linalg.norm(v) * np.linalg.norm(w) / abs(w @ v)
    return kap


def convdiff_eigs_kappa(N: int, beta):
    """Eigenvalues and condition numbers of the Kronecker-sum operator (the
    eigenvectors are Kronecker products, so the condition numbers multiply)."""
    lam = [factor_eigs(N, b) for b in beta]
    kap = [factor_kappa(N, b) for b in beta]
    L, K = lam[0], kap[0]
    for l2, k2 in zip(lam[1:], kap[1:]):
        L = (L[:, None] + l2[None, :]).ravel()
        K = (K[:, None] * k2[None, :]).ravel()
    return L, K
