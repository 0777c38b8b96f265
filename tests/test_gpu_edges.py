"""Edge cases of the GPU path: the largest Krylov dimension and sketch size the
kernels accept, the smallest parameters, and the degenerate inputs of the
method (an exact invariant subspace, the zero matrix).

Bars as in test_gpu_parity.py: the first steps against the oracle's first
steps to 1e-9 relative; the decomposition's identities (Krylov relation
16 m u, S = Omega U and sketch-orthonormality 1e-12) on the whole output.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2508_05400_amd as P
from oracle.rks import RKSOracle
from oracle.sketch import sketch_matrix
from workloads import CSR, convdiff2d, powerlaw_random

pytestmark = pytest.mark.gpu

U64 = 2.0**-53


def _extension(A, k, m, d, which, kind="sparse", seed=3):
    ctx = P.rks_create(A.row_ptr, A.col, A.val, A.n, k, m, d, which, 1e-10,
                       P.rks_opts_default(sketch_kind=kind, sketch_seed=seed, start_seed=1))
    try:
        P.rks_arnoldi(ctx, None)
        B = np.zeros((m + 1, m), order="F")
        S = np.zeros((d, m + 1), order="F")
        U = np.zeros((A.n, m + 1), order="F")
        assert P.rks_get_state(ctx, B, S, U) == m + 1
    finally:
        P.rks_destroy(ctx)
    return B, S, U


def _identities(A, B, S, U, m, d, kind, seed, rel_bar=None, orth_bar=1e-12):
    Sp = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    nA = abs(Sp).sum(axis=0).max()
    rel = np.linalg.norm(Sp @ U[:, :m] - U @ B) / (nA * np.linalg.norm(U[:, :m]))
    assert rel < (16 * m * U64 if rel_bar is None else rel_bar), rel
    om = sketch_matrix(A.n, d, kind, seed)
    OU = np.asarray(om @ U)
    assert np.linalg.norm(OU - S) < 1e-12
    assert np.linalg.norm(OU.T @ OU - np.eye(m + 1)) < orth_bar
    return nA


def test_largest_krylov_dimension_and_sketch(lib, cuda):
    """m = 255 (256 basis columns) and d = 1024, the kernels' limits: the
    least squares then runs from L2 (S is 2 MB) and the rotation uses its
    widest MFMA tiling."""
    A = powerlaw_random(3001, 4)
    k, m, d = 30, 255, 1024
    B, S, U = _extension(A, k, m, d, "LM")
    nA = _identities(A, B, S, U, m, d, "sparse", 3)
    o = RKSOracle(A, 1, 4, d, "LM", 1e-10, sketch="sparse", sketch_seed=3, start_seed=1)
    o.start(None)
    o.extend()
    assert np.abs(B[:5, :4] - o.B).max() <= 1e-9 * nA
    # a solve with these limits runs restarts (contraction, rotation of 256 columns)
    with P.Solver.from_csr(A, k=k, m=m, d=d, which="LM", tol=1e-10, sketch_seed=3, max_restarts=2) as s:
        assert s.solve() in (0, 1), P.rks_last_error(s.ctx)
        lam, X, res = s.eigpairs()
        assert np.all(np.isfinite(lam)) and np.all(np.isfinite(res))


def test_smallest_parameters(lib, cuda):
    """k = 1, m = k + 2, d = m + 1 (the smallest the checks allow), Gaussian sketch."""
    A = convdiff2d(9, (2.0, 1.0))
    k, m, d = 1, 3, 4
    B, S, U = _extension(A, k, m, d, "LR", kind="gauss", seed=5)
    _identities(A, B, S, U, m, d, "gauss", 5)
    # an isolated largest eigenvalue (200 against 1..80) converges within a few restarts
    D = _diag_csr(np.concatenate([np.arange(1.0, 81.0), [200.0]]))
    with P.Solver.from_csr(D, k=k, m=m, d=d, which="LR", tol=1e-10, sketch_kind="gauss", sketch_seed=5,
                           max_restarts=300) as s:
        assert s.solve() == 0, P.rks_last_error(s.ctx)
        lam, X, res = s.eigpairs()
    assert abs(lam[0] - 200.0) <= 1e-8 * 200.0
    assert res[0] <= 1e-8


def _diag_csr(d):
    n = len(d)
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.asarray(d, dtype=np.float64),
               {"kind": "diag"})


def _invariant_case():
    """A diagonal operator whose three largest eigenvalues (10, 9, 8) are
    isolated, and a start supported on their three coordinates: the Krylov
    space is that exact invariant subspace, so the remainder vanishes at
    column 3 (Section 2.1)."""
    n = 2000
    diag = np.concatenate([np.linspace(1.0, 2.0, n - 5), [10.0, 9.0, 8.0, 5.0, 4.0]])
    u0 = np.zeros(n)
    u0[[n - 5, n - 4, n - 3]] = [1.0, 2.0, -1.0]
    return _diag_csr(diag), diag, u0


@pytest.mark.parametrize("prec", ["fp64", "fp32+fx16"])
def test_exact_invariant_subspace_is_continued_past(lib, cuda, prec):
    """The extension meets the vanishing remainder at column 3, replaces it
    with the seeded tag-3 vector sketch-orthogonalised against U_3 and sets
    B(3, 2) = 0, as the oracle does: the whole decomposition equals the
    oracle's (entrywise 1e-9 ||A||_1) and satisfies the exact identities, and
    its Rayleigh quotient holds the three exact eigenvalues to 1e-12.  The
    pair basis meets the breakdown too (its first columns keep the start's
    three-coordinate support, so they span the invariant subspace exactly)
    and continues through the FP64 replacement vector like FP64 storage; its
    columns carry the pair rounding (relation to 64 * 2^-39; off the diagonal
    the sketch Gram matrix sees each stored column's rounding error against
    the others, about u (m+1) / sqrt(3 d) in norm with u = 2^-39, bar 4 times
    that) and agree with the oracle's pair storage to the same bars."""
    A, diag, u0 = _invariant_case()
    k, m, d = 5, 12, 40
    ctx = P.rks_create(A.row_ptr, A.col, A.val, A.n, k, m, d, "LM", 1e-10,
                       P.rks_opts_default(sketch_kind="sparse", sketch_seed=3, start_seed=1, precision=prec))
    try:
        P.rks_arnoldi(ctx, u0)
        B = np.zeros((m + 1, m), order="F")
        S = np.zeros((d, m + 1), order="F")
        U = np.zeros((A.n, m + 1), order="F")
        assert P.rks_get_state(ctx, B, S, U) == m + 1
    finally:
        P.rks_destroy(ctx)
    o = RKSOracle(A, k, m, d, "LM", 1e-10, sketch="sparse", sketch_seed=3, start_seed=1, store=prec)
    o.start(u0)
    o.extend()
    assert o.breakdowns == 1 and o.B[3, 2] == 0.0
    assert B[3, 2] == 0.0
    if prec == "fp64":
        nA = _identities(A, B, S, U, m, d, "sparse", 3)
    else:
        u = 2.0**-39
        nA = _identities(A, B, S, U, m, d, "sparse", 3, 64 * u, 4 * u * (m + 1) / np.sqrt(3 * d))
    assert np.abs(B - o.B).max() <= 1e-9 * nA, np.abs(B - o.B).max() / nA
    assert np.abs(U - o.U).max() <= 1e-9 * np.abs(o.U).max()
    ev = np.linalg.eigvals(B[:m, :m])
    for lam in (10.0, 9.0, 8.0):
        assert np.min(np.abs(ev - lam)) <= 1e-12 * lam


def test_breakdown_solve_matches_oracle(lib, cuda):
    """A whole solve through the breakdown: the exact pairs stay in the
    decomposition, the two further wanted pairs are found after it, and the
    five eigenvalues equal the oracle's (1e-10) and the exact ones."""
    A, diag, u0 = _invariant_case()
    k, m, d = 5, 12, 40
    ref = RKSOracle(A, k, m, d, "LM", 1e-10, sketch="sparse", sketch_seed=3, start_seed=1).run(u0)
    assert ref.converged
    with P.Solver.from_csr(A, k=k, m=m, d=d, which="LM", tol=1e-10, sketch_kind="sparse", sketch_seed=3,
                           start_seed=1) as s:
        assert s.solve(u0) == 0, P.rks_last_error(s.ctx)
        assert s.stats.breakdowns >= 1
        lam, X, res = s.eigpairs()
    assert np.max(np.abs(lam - ref.lam) / np.abs(ref.lam)) <= 1e-10
    assert np.max(np.abs(lam.real - np.array([10.0, 9.0, 8.0, 5.0, 4.0])) / 10.0) <= 1e-10
    assert res.max() <= 1e-8


def test_zero_matrix_reports_breakdown(lib, cuda):
    """The zero operator: the replacement vector's product with A vanishes
    too, so the continuation fails and the solver reports RKS_EBREAKDOWN."""
    n = 500
    A = _diag_csr(np.zeros(n))
    with P.Solver.from_csr(A, k=2, m=8, d=20, which="LM", tol=1e-10) as s:
        with pytest.raises(P.RksError) as ei:
            s.solve()
        assert ei.value.code == -6
        assert "replacement" in P.rks_last_error(s.ctx)
