"""Convection-diffusion operators  -Laplace(u) + beta . grad(u)  on the unit cube.

Central differences on a uniform grid with N interior points per axis,
h = 1/(N+1), homogeneous Dirichlet boundary, unknowns numbered x-fastest
(index = ix + N*iy + N^2*iz).  Along axis c the 1D factor is
h^-2 * tridiag(-1 - g_c, 2, -1 + g_c) with g_c = beta_c * h / 2, i.e. the
neighbour at ix-1 gets (-1 - g_c)/h^2 and the neighbour at ix+1 gets
(-1 + g_c)/h^2; the diagonal is 2*D/h^2.
"""
import numpy as np

from .csr import CSR


def _stencil(N: int, D: int, gammas, meta: dict) -> CSR:
    n = N ** D
    if n >= 2**31:
        raise ValueError("grid too large for int32 indices")
    h = 1.0 / (N + 1)
    ih2 = 1.0 / (h * h)
    idx = np.arange(n, dtype=np.int64)
    coords = [(idx // (N ** c)) % N for c in range(D)]
    offs, coefs, masks = [], [], []
    for c in reversed(range(D)):           # lower neighbours, farthest first
        g = gammas[c]
        offs.append(-(N ** c))
        coefs.append(np.broadcast_to((-1.0 - g) * ih2, (n,)))
        masks.append(coords[c] > 0)
    offs.append(0)
    coefs.append(np.full(n, 2.0 * D * ih2))
    masks.append(np.ones(n, dtype=bool))
    for c in range(D):                      # upper neighbours, nearest first
        g = gammas[c]
        offs.append(N ** c)
        coefs.append(np.broadcast_to((-1.0 + g) * ih2, (n,)))
        masks.append(coords[c] < N - 1)
    mask = np.stack(masks, axis=1)
    cols = idx[:, None] + np.asarray(offs, dtype=np.int64)[None, :]
    vals = np.stack(coefs, axis=1)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[mask].astype(np.int32)
    val = np.ascontiguousarray(vals[mask], dtype=np.float64)
    return CSR(n, row_ptr.astype(np.int32), col, val, meta)


def convdiff2d(N: int, beta=(20.0, 10.0)) -> CSR:
    """5-point operator on an N x N grid with constant velocity beta=(bx, by)."""
    h = 1.0 / (N + 1)
    g = [beta[0] * h / 2.0, beta[1] * h / 2.0]
    return _stencil(N, 2, g, {"kind": "convdiff2d", "N": N, "beta": tuple(map(float, beta))})


def convdiff3d(N: int, beta=(40.0, 20.0, 10.0)) -> CSR:
    """7-point operator on an N^3 grid with constant velocity beta=(bx, by, bz)."""
    h = 1.0 / (N + 1)
    g = [b * h / 2.0 for b in beta]
    return _stencil(N, 3, g, {"kind": "convdiff3d", "N": N, "beta": tuple(map(float, beta))})


def fourier_beta_field(N: int, seed: int, modes: int = 8, amp: float = 40.0, kmax: int = 3):
    """Velocity field made of random Fourier modes, sampled at the grid nodes.

    beta_c(x, y) = sum_q a_{c,q} cos(2 pi (p_q x + r_q y) + phi_{c,q}) for
    c in {x, y}, a ~ U(0, amp), integer wave vectors (p_q, r_q) uniform on
    [-kmax, kmax]^2 without (0, 0), phases ~ U(0, 2 pi).  Returns (bx, by),
    each an array of N*N node values in x-fastest order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    waves = []
    while len(waves) < modes:
        p, r = rng.integers(-kmax, kmax + 1, size=2)
        if p != 0 or r != 0:
            waves.append((int(p), int(r)))
    a = rng.uniform(0.0, amp, size=(2, modes))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(2, modes))
    h = 1.0 / (N + 1)
    t = (np.arange(N) + 1) * h
    x = np.tile(t, N)
    y = np.repeat(t, N)
    out = []
    for c in range(2):
        f = np.zeros(N * N)
        for q, (p, r) in enumerate(waves):
            f += a[c, q] * np.cos(2.0 * np.pi * (p * x + r * y) + phi[c, q])
        out.append(f)
    return out[0], out[1]


def convdiff2d_field(N: int, seed: int) -> CSR:
    """5-point operator on an N x N grid whose velocity is ``fourier_beta_field``."""
    bx, by = fourier_beta_field(N, seed)
    h = 1.0 / (N + 1)
    A = _stencil(N, 2, [bx * h / 2.0, by * h / 2.0],
                 {"kind": "convdiff2d_field", "N": N, "seed": int(seed)})
    return A
