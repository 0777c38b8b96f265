"""Counter-based random numbers for the sketch and the start vector (oracle side).

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4x32-bit counter and
a 2x32-bit key, ten rounds, the key bumped by the Weyl constants between
rounds.  Pinned by the published known-answer vectors (tests/golden).

Stream layout used by the solver (written spec, implemented independently by
the GPU library):
  counter = (i mod 2^32, i div 2^32, c2, tag), key = (seed mod 2^32, seed div 2^32)
  tag 0: Gaussian embedding, c2 = row-pair index  -> one Box-Muller pair
  tag 1: sparse-sign embedding, c2 in {0, 1}      -> 8 words for column i
  tag 2: start vector, c2 = 0                     -> entry i = first Box-Muller output
  tag 3: breakdown replacement vector, c2 = breakdown count
A uniform in the open interval (0, 1) is ((hi << 20) | (lo >> 12)) + 0.5 scaled by
2^-52: 52 random bits plus one half, exact in FP64 (with 53 bits the top value
would round to 1.0).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)

TAG_GAUSS, TAG_SPARSE, TAG_START, TAG_BREAK = 0, 1, 2, 3


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Apply Philox4x32-10 to counters (arrays of uint32-valued ints) under key
    (k0, k1).  Returns four uint64 arrays holding the 32-bit output words."""
    c = [np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3)]
    c = np.broadcast_arrays(*c)
    c = [x.copy() for x in c]
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return c


def uniform01(hi, lo):
    """Uniform double in the open interval (0, 1) from two 32-bit words."""
    hi = np.asarray(hi, dtype=np.uint64)
    lo = np.asarray(lo, dtype=np.uint64)
    x = (hi << np.uint64(20)) | (lo >> np.uint64(12))
    return (x.astype(np.float64) + 0.5) * 2.0**-52


def box_muller(u1, u2):
    """Two independent N(0,1) values from two uniforms in (0, 1)."""
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def _split(i):
    i = np.asarray(i, dtype=np.uint64)
    return i & _MASK, i >> np.uint64(32)


def _key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def gaussian_pair(i, pair, tag, seed):
    """Box-Muller pair for counter (i, pair, tag) under ``seed``."""
    lo, hi = _split(i)
    w = philox4x32_10(lo, hi, pair, tag, *_key(seed))
    return box_muller(uniform01(w[0], w[1]), uniform01(w[2], w[3]))


def start_vector(n: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) start vector: entry i is the first Box-Muller output of
    counter (i, 0, tag 2)."""
    g0, _ = gaussian_pair(np.arange(n, dtype=np.uint64), 0, TAG_START, seed)
    return g0


def breakdown_vector(n: int, seed: int, count: int) -> np.ndarray:
    """Seeded N(0,1) vector used to continue after an exact invariant subspace."""
    g0, _ = gaussian_pair(np.arange(n, dtype=np.uint64), count, TAG_BREAK, seed)
    return g0
