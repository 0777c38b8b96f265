"""Random non-symmetric sparse matrix with power-law row lengths."""
import numpy as np

from .csr import CSR, from_triplets


def _mean_len(alpha: float, lmin: int, lmax: int) -> float:
    ell = np.arange(lmin, lmax + 1, dtype=np.float64)
    w = ell ** (-alpha)
    return float((ell * w).sum() / w.sum())


def powerlaw_exponent(mean: float = 16.0, lmin: int = 4, lmax: int = 512) -> float:
    """Exponent alpha of P(L = l) ~ l^-alpha on [lmin, lmax] whose mean is ``mean``."""
    lo, hi = 0.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _mean_len(mid, lmin, lmax) > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def powerlaw_random(n: int, seed: int, mean_len: float = 16.0, lmin: int = 4,
                    lmax: int = 512, diag_std: float = 0.1) -> CSR:
    """Row i holds L_i off-diagonal entries in distinct uniform random columns
    (L_i drawn from the power law above) with values N(0,1)/sqrt(L_i), plus a
    diagonal entry N(0, diag_std^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    alpha = powerlaw_exponent(mean_len, lmin, lmax)
    ell = np.arange(lmin, min(lmax, n - 1) + 1)
    p = ell.astype(np.float64) ** (-alpha)
    p /= p.sum()
    L = rng.choice(ell, size=n, p=p).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), L)
    cols = rng.integers(0, n, size=rows.size, dtype=np.int64)
    # Redraw until every row has distinct off-diagonal columns.
    for _ in range(100):
        key = rows * n + cols
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        bad = np.zeros(rows.size, dtype=bool)
        bad[order[dup]] = True
        bad |= cols == rows
        if not bad.any():
            break
        cols[bad] = rng.integers(0, n, size=int(bad.sum()), dtype=np.int64)
    else:  # pragma: no cover - astronomically unlikely
        raise RuntimeError("could not draw distinct columns")
    vals = rng.standard_normal(rows.size) / np.sqrt(L[rows].astype(np.float64))
    drow = np.arange(n, dtype=np.int64)
    dval = diag_std * rng.standard_normal(n)
    A = from_triplets(n, np.concatenate([rows, drow]), np.concatenate([cols, drow]),
                      np.concatenate([vals, dval]),
                      {"kind": "powerlaw_random", "n": n, "seed": int(seed),
                       "alpha": alpha, "lmin": lmin, "lmax": lmax})
    return A
