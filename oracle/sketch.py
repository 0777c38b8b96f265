"""The random embedding Omega in R^{d x n}, built explicitly (oracle side).

Oblivious subspace embeddings (Section 2, "Preliminaries"): either a dense
matrix of normalised Gaussian entries, or a sparse-sign matrix with zeta
nonzeros +-1/sqrt(zeta) per column (Section 5 uses zeta = 8).

Readings where the paper is open:
  * Gaussian entries are N(0, 1/d), so that E||Omega x||^2 = ||x||^2.
  * Sparse-sign scaling is 1/sqrt(zeta) (unit columns).  The paper writes
    1/sqrt(d); Ritz values and residual estimates are invariant under
    Omega -> c*Omega, so the choice does not change the method's output.
  * The zeta rows of a column are distinct, chosen by Floyd's sampling
    algorithm: draw t = 0..zeta-1 takes j = d - zeta + t and
    v = floor(r_t * (j + 1) / 2^32) in [0, j]; it adds v, or j if v is already
    taken.  Draw t's sign is negative iff bit 0 of r_t is set.  The words
    r_0..r_7 are Philox4x32-10 outputs of counters (i, 0, tag 1) and (i, 1, tag 1).
  * Gaussian entry (b, i) is output (b mod 2) of the Box-Muller pair of
    counter (i, floor(b / 2), tag 0).
"""
import numpy as np
import scipy.sparse as sp

from .philox import philox4x32_10, gaussian_pair, _split, _key, TAG_GAUSS, TAG_SPARSE


def sparse_sign_columns(cols, d: int, zeta: int, seed: int):
    """Rows (len(cols) x zeta, int) and signs (+-1.0) of the given columns."""
    if not (1 <= zeta <= 8 and zeta <= d):
        raise ValueError("need 1 <= zeta <= min(8, d)")
    lo, hi = _split(np.asarray(cols, dtype=np.uint64))
    k0, k1 = _key(seed)
    words = philox4x32_10(lo, hi, 0, TAG_SPARSE, k0, k1) + philox4x32_10(lo, hi, 1, TAG_SPARSE, k0, k1)
    nc = lo.size
    rows = np.empty((nc, zeta), dtype=np.int64)
    signs = np.empty((nc, zeta))
    for t in range(zeta):
        j = d - zeta + t
        r = words[t]
        v = ((r * np.uint64(j + 1)) >> np.uint64(32)).astype(np.int64)
        taken = np.zeros(nc, dtype=bool)
        for s in range(t):
            taken |= rows[:, s] == v
        rows[:, t] = np.where(taken, j, v)
        signs[:, t] = np.where((r & np.uint64(1)) == 1, -1.0, 1.0)
    return rows, signs


def sketch_matrix(n: int, d: int, kind: str, seed: int, zeta: int = 8):
    """Explicit Omega: a dense ndarray (Gaussian) or a CSC sparse matrix (sparse-sign)."""
    if kind == "gauss":
        om = np.empty((d, n))
        i = np.arange(n, dtype=np.uint64)
        for p in range((d + 1) // 2):
            g0, g1 = gaussian_pair(i, p, TAG_GAUSS, seed)
            om[2 * p] = g0
            if 2 * p + 1 < d:
                om[2 * p + 1] = g1
        return om / np.sqrt(d)
    if kind == "sparse":
        rows, signs = sparse_sign_columns(np.arange(n), d, zeta, seed)
        cols = np.repeat(np.arange(n), zeta)
        return sp.csc_matrix((signs.ravel() / np.sqrt(zeta), (rows.ravel(), cols)), shape=(d, n))
    raise ValueError(f"unknown sketch kind {kind!r}")
