"""Randomized Krylov-Schur in plain FP64 (oracle side).

Follows Algorithm 1 (rKS) and Algorithm 2 (extension of an rKS factorisation)
of the paper in their order, with:
  * the sketch S = Omega U stored and truncated without re-sketching
    (Section 3.1, after Algorithm 2);
  * residual estimates |b^T y| / |lambda| (Section 4.1, eq. "rks_reserror_bound");
  * locking of converged leading Schur vectors, which stay as the leading
    basis columns so every new vector is sketch-orthogonalised against them
    (Sections 4.2-4.4, deflated operator of eq. "AqSchurDeflatedSubspace");
  * whitening re-orthogonalisation U <- U R^-1 from a Householder QR of the
    sketch (Section 3.3).

Small dense steps use LAPACK through SciPy: dgees (real Schur form),
dtrexc (Bai-Demmel reordering of adjacent blocks), dgeev (eigenpairs of the
truncated factor), Householder QR (dgeqrf) for the least-squares problems.

Readings where the paper is open (listed with the reasons in the design notes):
  * which: LM |lambda| largest, SM smallest, LR Re largest, SR Re smallest;
    ties broken by larger imaginary part; the wanted eigenvalues are moved to
    the front one block at a time in that priority order; if the k-th and
    (k+1)-th form a conjugate pair both are kept (effective k = k+1).
  * least squares h = S_j^+ z: Householder QR of S_j.
  * locking: leading position i (a 1x1 or 2x2 diagonal block) is locked when
    every |b_i| of the block is <= tol * max(|lambda_block|, u ||T||_F);
    locking stops at the first position that fails.
  * whitening when ||S_k^T S_k - I||_F > whiten_tol (default 1e-12).
  * breakdown (an invariant subspace): when beta <= 1e-12 ||Omega w|| the new
    vector is replaced by a seeded random vector sketch-orthogonalised against
    U_j, and B(j+1, j) is set to 0.
  * convergence: all effective-k estimates <= tol (or, with resid_tol > 0,
    every wanted pair's FP64 residual <= resid_tol); at most max_restarts
    contraction/extension cycles after the first extension.
  * restart size keep (Algorithm 1 truncates to k): any leading truncation is
    again an rKS decomposition (Section 3.1); keep = -1 takes
    k + (m - k) // 4, at most m - 2.

Pins (tests/test_oracle_pins.py): the decomposition's identities through
restarts, textbook Arnoldi for Omega = I, closed-form convection-diffusion
spectra, dense brute force, the Section 4.1 residual bound, breakdown
recovery, whitening of a decomposition with a non-orthonormal sketch,
scale invariance.  Parity unpinned: the eigenvalues it returns for
strongly non-normal operators (condition numbers 1e11-1e13, as on the 1000^2
smallest-real-part workload) have no reference at that accuracy; only their
residuals are checked there.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.linalg import lapack

from .philox import start_vector, breakdown_vector
from .sketch import sketch_matrix

UNIT_ROUNDOFF = 2.0**-53
BREAKDOWN_REL = 1e-12


def round_storage(x, store):
    """Round FP64 values to a basis storage format, to nearest with ties to
    even: 'fp64' leaves them, 'fp32' rounds to binary32, 'bf16' rounds to
    binary32 and then to bfloat16 (binary32's sign and exponent with an 8-bit
    significand).  The bfloat16 step is written out from the definition: the
    two neighbouring bfloat16 values bracket the binary32 value, the nearer
    one is taken, and a tie goes to the one whose last significand bit is 0.
    'fp32+bf16' stores a pair: hi, the binary32 rounding, and lo, the bfloat16
    rounding (as above) of the remainder x - hi, which FP64 holds exactly; the
    stored value is hi + lo, within 2^-32 |x| of x.
    'fp32+fx16' stores hi and a 16-bit signed integer q: the remainder x - hi
    measured in units of 2^-15 ulp(hi) and rounded to the nearest integer
    (ties to even), where ulp(hi) = 2^(max(e, 1) - 150) for the biased
    binary32 exponent e of hi (the spacing of binary32 values at hi).  Since
    |x - hi| <= ulp(hi) / 2, |q| <= 2^14; the stored value hi + q 2^-15 ulp(hi)
    is within 2^-16 ulp(hi) <= 2^-39 |hi| of x."""
    x = np.asarray(x, dtype=np.float64)
    if store == "fp64":
        return x.copy()
    if store == "fp32+bf16":
        hi = round_storage(x, "fp32")
        return hi + round_storage(x - hi, "bf16")
    if store == "fp32+fx16":
        hi, q, step = fx16_pair(x)
        return hi + q * step
    x32 = x.astype(np.float32)
    if store == "fp32":
        return x32.astype(np.float64)
    if store != "bf16":
        raise ValueError(f"unknown storage format {store!r}")
    bits = x32.view(np.uint32)
    down = (bits & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)   # toward zero
    up_bits = (bits & np.uint32(0xFFFF0000)) + np.uint32(0x10000)               # next magnitude
    up = up_bits.view(np.float32).astype(np.float64)
    v = x32.astype(np.float64)
    dd, du = np.abs(v - down), np.abs(up - v)
    down_even = ((bits >> np.uint32(16)) & np.uint32(1)) == 0
    take_up = (du < dd) | ((du == dd) & ~down_even & (dd > 0))
    return np.where(take_up, up, down)


def fx16_pair(x):
    """The parts of the 'fp32+fx16' storage of x (see round_storage): hi (as
    FP64), the integer q (as FP64) and the unit step = 2^-15 ulp(hi)."""
    x = np.asarray(x, dtype=np.float64)
    hi32 = x.astype(np.float32)
    hi = hi32.astype(np.float64)
    e = ((hi32.view(np.uint32) >> np.uint32(23)) & np.uint32(0xFF)).astype(np.int64)
    step = np.ldexp(1.0, np.maximum(e, 1) - 150 - 15)
    q = np.rint((x - hi) / step)    # exact quotient (a power of two); rint ties to even
    return hi, q, step


def which_key(lam: complex, which: str):
    """Sort key, larger = more wanted (ties: larger imaginary part first)."""
    lam = complex(lam)
    if which == "LM":
        return (abs(lam), lam.imag)
    if which == "SM":
        return (-abs(lam), lam.imag)
    if which == "LR":
        return (lam.real, lam.imag)
    if which == "SR":
        return (-lam.real, lam.imag)
    raise ValueError(f"unknown which {which!r}")


def _blocks(T: np.ndarray, start: int = 0):
    """Diagonal blocks (position, size, eigenvalue with Im >= 0) of a
    quasi-triangular T from ``start`` on."""
    n = T.shape[0]
    out = []
    i = start
    while i < n:
        if i + 1 < n and T[i + 1, i] != 0.0:
            blk = T[i:i + 2, i:i + 2]
            ev = np.linalg.eigvals(blk)
            lam = ev[0] if ev[0].imag >= ev[1].imag else ev[1]
            out.append((i, 2, complex(lam)))
            i += 2
        else:
            out.append((i, 1, complex(T[i, i])))
            i += 1
    return out


def order_wanted(T: np.ndarray, Z: np.ndarray, which: str, kw: int):
    """Move the kw most wanted eigenvalues of the real Schur form (T, Z) to the
    leading positions, most wanted first.  Returns (T, Z, p) where p = kw, or
    kw + 1 when a conjugate pair straddles the boundary."""
    T = np.array(T, order="F")
    Z = np.array(Z, order="F")
    pos = 0
    n = T.shape[0]
    while pos < kw and pos < n:
        blks = _blocks(T, pos)
        best = max(blks, key=lambda b: which_key(b[2], which))
        if best[0] != pos:
            T, Z, info = lapack.dtrexc(T, Z, best[0] + 1, pos + 1)
            if info != 0:
                raise RuntimeError(f"dtrexc rejected a swap (info={info})")
        size = 2 if pos + 1 < n and T[pos + 1, pos] != 0.0 else 1
        pos += size
    return T, Z, pos


@dataclass
class OracleResult:
    lam: np.ndarray          # effective-k Ritz values, sorted by `which`
    X: np.ndarray            # n x keff Ritz vectors, LAPACK real packing, unit 2-norm
    resid: np.ndarray        # ||A x - lam x|| / (||A||_1 ||x||)
    est: np.ndarray          # paper's estimates |b^T y| / |lam| at exit
    converged: bool
    restarts: int
    matvecs: int
    locked: int
    history: list = field(default_factory=list)   # max estimate after each contraction


class RKSOracle:
    """State of an rKS run: U (n x (m+1)), S = Omega U, B ((m+1) x m)."""

    def __init__(self, A, k, m, d, which="LM", tol=1e-10, sketch="sparse", zeta=8,
                 sketch_seed=0, start_seed=1, lock=True, whiten_tol=1e-12,
                 max_restarts=300, keep=None, resid_tol=0.0,
                 store="fp64"):
        if hasattr(A, "row_ptr"):
            A = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
        self.A = sp.csr_matrix(A, dtype=np.float64)
        n = self.A.shape[0]
        if not (1 <= k and k + 2 <= m and m + 1 <= d and d <= n and m + 1 <= n):
            raise ValueError("need 1 <= k, k+2 <= m, m+1 <= d <= n")
        if keep == -1:      # automatic: k + (m - k) / 4, at most m - 2
            keep = max(k, min(k + (m - k) // 4, m - 2))
        keep = k if not keep else keep
        if not (k <= keep <= m - 2):
            raise ValueError("need k <= keep <= m-2")
        self.n, self.k, self.m, self.d = n, k, m, d
        # restart size: any leading truncation of an rKS decomposition is one
        # (Section 3.1); Algorithm 1 keeps k, a larger keep keeps more of the
        # most wanted Schur vectors.  Only the leading k are tested/returned.
        self.keep = keep
        self.which, self.tol, self.lock = which, tol, lock
        self.whiten_tol, self.max_restarts = whiten_tol, max_restarts
        # > 0: also stop once every wanted pair's FP64 residual
        # ||A x - lambda x|| / (||A||_1 ||x||) is <= resid_tol (checked after
        # every contraction)
        self.resid_tol = resid_tol
        # storage format of the basis: 'fp64', or 'fp32' / 'bf16' for the
        # low-precision pattern (the product with A then runs on binary32
        # copies of A's values and its result is rounded to binary32; the
        # stored column is the unnormalised remainder rounded to the format,
        # its scale 1/beta is kept in FP64, and the sketch is taken of the
        # stored value); 'fp32+bf16' and 'fp32+fx16' store the remainder as
        # such a pair and form the product with A in FP64 from the stored value
        self.store = store
        if store != "fp64":
            self.A_low = sp.csr_matrix((round_storage(self.A.data, "fp32"), self.A.indices, self.A.indptr),
                                       shape=self.A.shape)
            self.stored = np.zeros((self.A.shape[0], m + 1))   # stored values v_j
            self.cs = np.zeros(m + 1)                          # u_j = cs_j v_j
        self.start_seed = start_seed
        self.Om = sketch_matrix(n, d, sketch, sketch_seed, zeta)
        self.normA1 = float(abs(self.A).sum(axis=0).max())
        self.U = np.zeros((n, m + 1))
        self.S = np.zeros((d, m + 1))
        self.B = np.zeros((m + 1, m))
        self.j = 0          # index of the last basis column
        self.q = 0          # number of locked columns
        self.keff = 0
        self.kr = 0         # wanted pairs: leading k, k+1 when a 2x2 block straddles k
        self.matvecs = 0
        self.breakdowns = 0
        self.whitenings = 0

    # -- sketch --------------------------------------------------------------
    def sketch(self, x):
        return np.asarray(self.Om @ x).ravel()

    # -- start (Algorithm 2 with no initial decomposition) -------------------
    def start(self, u0=None):
        ut = start_vector(self.n, self.start_seed) if u0 is None else np.asarray(u0, dtype=np.float64)
        ut = round_storage(ut, self.store)
        s = self.sketch(ut)
        nrm = np.linalg.norm(s)
        self._set_column(0, ut, nrm)
        self.S[:, 0] = s / nrm
        self.j = 0

    # -- least squares with the stored sketch ------------------------------
    @staticmethod
    def lstsq(Sj, z):
        """h = argmin ||S_j h - z||_2 by Householder QR of S_j."""
        Qs, Rs = np.linalg.qr(Sj, mode="reduced")
        return sla.solve_triangular(Rs, Qs.T @ z)

    # -- Algorithm 2 ---------------------------------------------------------
    def _set_column(self, j, v, scale):
        """u_j = v / scale (with a low-precision basis v is the stored value
        and 1/scale its FP64 scale)."""
        if self.store == "fp64":
            self.U[:, j] = v / scale
        else:
            self.stored[:, j] = v
            self.cs[j] = 1.0 / scale
            self.U[:, j] = v * self.cs[j]

    def apply(self, j):
        """A u_j.  With a low-precision basis, u_j = c_j v_j is a stored
        vector v_j times its FP64 scale c_j: the product A v_j is formed from
        binary32 copies of A's values and rounded to binary32, then scaled
        (the pairs 'fp32+bf16' and 'fp32+fx16': in FP64 from A's values and
        the stored value)."""
        if self.store == "fp64":
            return self.A @ self.U[:, j]
        if self.store in ("fp32+bf16", "fp32+fx16"):
            return self.cs[j] * (self.A @ self.stored[:, j])
        w = round_storage(self.A_low @ self.stored[:, j], "fp32")
        return self.cs[j] * w

    def _new_direction(self, j, v):
        """Sketched Gram-Schmidt of v against the first j+1 columns: the
        coefficients h solve min ||S_j h - Omega v|| and the remainder
        v - U_j h is returned with its sketch (taken from the remainder
        itself, not updated from the sketches)."""
        h = self.lstsq(self.S[:, :j + 1], self.sketch(v))
        rem = round_storage(v - self.U[:, :j + 1] @ h, self.store)
        return h, rem, self.sketch(rem)

    def extend(self):
        """Algorithm 2: grow the sketch-orthonormal Krylov decomposition
        A U_m = U_{m+1} B from j+1 to m+1 columns.  Column j+1 is the
        remainder of A u_j after the sketched projection onto U_j, scaled to a
        unit sketch; its scale is the subdiagonal entry of B.  A remainder
        whose sketch vanishes against that of A u_j (an invariant subspace,
        Section 2.1) is replaced by a seeded random direction treated the same
        way, with a zero subdiagonal entry."""
        for j in range(self.j, self.m):
            Au = self.apply(j)
            self.matvecs += 1
            h, rem, srem = self._new_direction(j, Au)
            self.B[:j + 1, j] = h
            scale = np.linalg.norm(srem)
            sub = scale
            if scale <= BREAKDOWN_REL * np.linalg.norm(self.sketch(Au)):
                self.breakdowns += 1
                r = breakdown_vector(self.n, self.start_seed, self.breakdowns)
                _, rem, srem = self._new_direction(j, r)
                scale = np.linalg.norm(srem)
                sub = 0.0
            self._set_column(j + 1, rem, scale)
            self.S[:, j + 1] = srem / scale
            self.B[j + 1, j] = sub
        self.j = self.m

    # -- Algorithm 1, contraction -------------------------------------------
    def contract(self):
        """Schur form of the active block, reorder the wanted eigenvalues to the
        front, truncate.  Leaves an rKS decomposition of order keff."""
        m, q, k = self.m, self.q, self.k
        B = self.B
        T_a, Z = sla.schur(B[q:m, q:m], output="real")
        T_a, Z, p = order_wanted(T_a, Z, self.which, self.keep - q)
        keff = q + p
        kr = min(k, keff)
        if q < kr < keff and T_a[kr - q, kr - 1 - q] != 0.0:
            kr += 1
        self.kr = kr
        if self.lock == 2:
            T_a, Z = self._front_converged(T_a, Z, B[m, q:m], kr - q)
        Q = np.eye(m)
        Q[q:, q:] = Z
        T = np.zeros((m, m))
        T[:q, :q] = B[:q, :q]
        T[:q, q:] = B[:q, q:m] @ Z
        T[q:, q:] = T_a
        b = B[m, :m] @ Q
        Unew = self.U[:, :m] @ Q[:, :keff]
        Snew = self.S[:, :m] @ Q[:, :keff]
        self.U[:, :keff] = Unew
        self.S[:, :keff] = Snew
        self.U[:, keff] = self.U[:, m]
        self.S[:, keff] = self.S[:, m]
        self.U[:, keff + 1:] = 0.0
        self.S[:, keff + 1:] = 0.0
        Tk = T[:keff, :keff].copy()
        bk = b[:keff].copy()
        # whitening (Section 3.3)
        Sk = self.S[:, :keff]
        if np.linalg.norm(Sk.T @ Sk - np.eye(keff)) > self.whiten_tol:
            Tk, bk = self.whiten(Tk, bk)
        if self.store != "fp64":
            # the rotated columns and u_{k+1} are stored rounded with scale 1;
            # S keeps the FP64 truncated sketch (not re-sketched)
            self.U[:, :keff + 1] = round_storage(self.U[:, :keff + 1], self.store)
            self.stored[:] = 0.0
            self.stored[:, :keff + 1] = self.U[:, :keff + 1]
            self.cs[:] = 0.0
            self.cs[:keff + 1] = 1.0
        self.B[:] = 0.0
        self.B[:keff, :keff] = Tk
        self.B[keff, :keff] = bk
        self.keff = keff
        self.j = keff

    def whiten(self, Tk, bk):
        """Section 3.3: with S_k = Q_s R (thin QR), the decomposition
        A U_k = U_k T + u bT is equivalent to one in U_k R^-1, whose sketch is
        Q_s (orthonormal): T becomes R T R^-1 and bT becomes bT R^-1.
        Updates U and S in place and returns the new (T, b)."""
        keff = Tk.shape[0]
        Qs, R = np.linalg.qr(self.S[:, :keff], mode="reduced")
        Rinv = sla.solve_triangular(R, np.eye(keff))
        self.U[:, :keff] = self.U[:, :keff] @ Rinv
        self.S[:, :keff] = Qs
        self.whitenings += 1
        return R @ Tk @ Rinv, bk @ Rinv

    def _front_converged(self, T, Z, b_row, nw):
        """Aggressive deflation (Section 4.4, after the deflation theorem): the
        decomposition may be reordered to test other Schur vectors for locking.
        Walk the nw wanted positions of the active Schur form (T, Z) in order;
        a block whose b entries pass the locking test once it is moved to the
        front of the active part (b = b_row Z after the move) is moved there, so
        that the leading-block locking then takes it.  The others keep their
        order behind the moved ones."""
        tn = np.linalg.norm(T[:nw, :nw])
        pos, idx = 0, 0
        while idx < nw:
            s = 2 if idx + 1 < T.shape[0] and T[idx + 1, idx] != 0.0 else 1
            if idx == pos:
                Tc, Zc = T, Z
            else:
                Tc, Zc, info = lapack.dtrexc(np.array(T, order="F"), np.array(Z, order="F"), idx + 1, pos + 1)
                if info != 0:
                    idx += s
                    continue
            sn = 2 if pos + 1 < Tc.shape[0] and Tc[pos + 1, pos] != 0.0 else 1
            lam = np.linalg.eigvals(Tc[pos:pos + sn, pos:pos + sn])
            bl = b_row @ Zc[:, pos:pos + sn]
            if np.all(np.abs(bl) <= self.tol * max(np.max(np.abs(lam)), UNIT_ROUNDOFF * tn)):
                T, Z = Tc, Zc
                pos += sn
            idx += s
        return T, Z

    def ritz(self):
        """Eigenpairs of the wanted leading block T_k and the estimates
        |b^T y| / |lambda| (Section 4.1)."""
        keff, kr = self.keff, self.kr
        Tk = self.B[:kr, :kr]
        bk = self.B[keff, :kr]
        lam, Y = sla.eig(Tk)
        with np.errstate(divide="ignore", invalid="ignore"):
            est = np.abs(bk @ Y) / np.abs(lam)
        return lam, Y, est

    def lock_converged(self):
        """Extend the locked set over leading blocks whose b entries are small
        relative to the block's eigenvalue (Section 4.4), and zero them."""
        keff = self.keff
        Tk = self.B[:keff, :keff]
        bk = self.B[keff, :keff]
        tnorm = np.linalg.norm(Tk)
        q = self.q
        for (i, s, lam) in _blocks(Tk, q):
            if i != q or i + s > self.kr:
                break
            scale = max(abs(lam), UNIT_ROUNDOFF * tnorm)
            if np.all(np.abs(bk[i:i + s]) <= self.tol * scale):
                q = i + s
            else:
                break
        self.B[keff, :q] = 0.0
        self.q = q

    def run(self, u0=None):
        self.start(u0)
        self.extend()
        history = []
        restarts = 0
        while True:
            self.contract()
            lam, Y, est = self.ritz()
            history.append(float(np.max(est)))
            converged = bool(np.all(est <= self.tol))
            if not converged and self.resid_tol > 0.0:
                X = self.U[:, :self.kr] @ Y
                R = self.A @ X - X * lam[None, :]
                res = np.linalg.norm(R, axis=0) / (self.normA1 * np.linalg.norm(X, axis=0))
                converged = bool(np.all(res <= self.resid_tol))
            if converged or restarts >= self.max_restarts:
                break
            if self.lock:
                self.lock_converged()
            self.extend()
            restarts += 1
        return self._finish(converged, restarts, history)

    def _finish(self, converged, restarts, history):
        keff, kr = self.keff, self.kr
        Tk = self.B[:kr, :kr]
        bk = self.B[keff, :kr]
        lam, Y = sla.eig(Tk)
        with np.errstate(divide="ignore", invalid="ignore"):
            est = np.abs(bk @ Y) / np.abs(lam)
        lam, X, resid, est = eigpairs(self.A, self.U[:, :kr], lam, Y, est, self.which, self.normA1)
        return OracleResult(lam, X, resid, est, converged, restarts, self.matvecs, self.q, history)


def eigpairs(A, Uk, lam, Y, est, which, normA1):
    """Ritz vectors x = U_k y sorted by ``which``, packed as LAPACK does (a
    conjugate pair occupies two columns: real and imaginary part of the
    member with positive imaginary part), each of unit 2-norm, with the
    relative residual ||A x - lambda x||_2 / (||A||_1 ||x||_2)."""
    order = sorted(range(len(lam)), key=lambda i: which_key(lam[i], which), reverse=True)
    lam = lam[order]
    Y = Y[:, order]
    est = est[order]
    n = Uk.shape[0]
    X = np.zeros((n, len(lam)))
    resid = np.zeros(len(lam))
    i = 0
    while i < len(lam):
        x = Uk @ Y[:, i]
        x = x / np.linalg.norm(x)
        r = A @ x - lam[i] * x
        res = np.linalg.norm(r) / normA1
        if abs(lam[i].imag) > 0 and i + 1 < len(lam):
            X[:, i] = x.real
            X[:, i + 1] = x.imag
            resid[i] = resid[i + 1] = res
            i += 2
        else:
            X[:, i] = x.real
            resid[i] = res
            i += 1
    return lam, X, resid, est


def rks(A, k, m, d, which="LM", tol=1e-10, u0=None, **kw):
    """Run the oracle rKS to convergence (or max_restarts); see RKSOracle."""
    return RKSOracle(A, k, m, d, which, tol, **kw).run(u0)


def ks_oracle(A, k, m, which="LM", tol=1e-10, **kw):
    """Deterministic Krylov-Schur, the paper's point of comparison: the same
    algorithm with Omega = I, so the sketched inner product is the Euclidean
    one, S = U, and the least squares h = U^+ w is the orthogonal projection
    (the special case noted with Algorithm 2; pinned against textbook
    Arnoldi in the oracle's tests)."""
    if hasattr(A, "row_ptr"):
        A = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    n = A.shape[0]
    o = RKSOracle(A, k, m, m + 1, which, tol, **kw)
    o.Om = sp.identity(n, format="csr")
    o.d = n
    o.S = np.zeros((n, m + 1))
    return o
