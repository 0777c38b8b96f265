"""Synthetic tridiagonal family of Section 5.1 (Table "SynthTestMatrices").

The diagonal carries f(t_i) on n equispaced points t_i in [2, 10]; both
off-diagonals are independent N(0,1)/100 noise (eq. "synthMathSubdiags").
"""
import numpy as np

from .csr import CSR

SPECTRA = {
    "exponential": lambda t: np.exp(t / 10.0),
    "logarithmic": lambda t: np.log(t + 1.0),
    "harmonic": lambda t: 1.0 + 1.0 / t**2,
    "geometric": lambda t: 0.99**t,
}


def tridiag_noisy(n: int, spectrum: str, seed: int) -> CSR:
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.linspace(2.0, 10.0, n)
    diag = SPECTRA[spectrum](t)
    sub = rng.standard_normal(n - 1) / 100.0   # A[i+1, i]
    sup = rng.standard_normal(n - 1) / 100.0   # A[i, i+1]
    counts = np.full(n, 3, dtype=np.int64)
    counts[0] -= 1
    counts[-1] -= 1
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.empty(row_ptr[-1], dtype=np.int32)
    val = np.empty(row_ptr[-1])
    pos = row_ptr[:-1].copy()
    i = np.arange(n)
    m = i > 0
    col[pos[m]] = i[m] - 1
    val[pos[m]] = sub
    pos[m] += 1
    col[pos] = i
    val[pos] = diag
    pos += 1
    m = i < n - 1
    col[pos[m]] = i[m] + 1
    val[pos[m]] = sup
    return CSR(n, row_ptr.astype(np.int32), col, val,
               {"kind": "tridiag_noisy", "n": n, "spectrum": spectrum, "seed": int(seed)})
