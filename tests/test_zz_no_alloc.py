"""The no-allocation sketch entry point against rks_sketch on a context with
the same embedding: two calls in a row (the second with a smaller input),
both sketch kinds, through the C-ABI.  Both run the same kernels on the same
grid, so the results agree to the bit; the bar of the other sketch checks
(64 u sum |Omega_bi x_i| against the oracle's explicit Omega) is asserted
as well."""
import numpy as np
import pytest

import paper_2508_05400_amd as P
from oracle.sketch import sketch_matrix
from workloads import convdiff2d, start_vector_normal

pytestmark = pytest.mark.gpu

U64 = 2.0**-53


def _ctx_sketch(cuda, n, d, kind, zeta, seed, x):
    A = convdiff2d(int(round(np.sqrt(n))), (2.0, 1.0))
    assert A.n == n
    ctx = P.rks_create(A.row_ptr, A.col, A.val, A.n, 2, min(20, d - 1), d, "LM", 1e-10,
                       P.rks_opts_default(sketch_kind=kind, zeta=zeta, sketch_seed=seed))
    try:
        z = cuda.zeros(d, dtype=cuda.float64, device="cuda")
        P.rks_sketch(ctx, x, z)
        return z.cpu().numpy()
    finally:
        P.rks_destroy(ctx)


@pytest.mark.parametrize("kind,zeta", [("sparse", 8), ("gauss", 8), ("sparse", 3)])
def test_noalloc_sketch_matches_context_sketch(lib, cuda, kind, zeta):
    seed = 17
    for side, d in ((300, 700), (61, 130)):   # second call: smaller n and d
        n = side * side
        xh = start_vector_normal(n, side)
        x = cuda.from_numpy(xh).cuda()
        ref = _ctx_sketch(cuda, n, d, kind, zeta, seed, x)
        z = cuda.full((d,), float("nan"), dtype=cuda.float64, device="cuda")
        print(f"noalloc sketch kind={kind} zeta={zeta} n={n} d={d}", flush=True)
        P.rks_sketch_noalloc(n, d, kind, zeta, seed, x, z, cuda.cuda.current_stream())
        cuda.cuda.synchronize()
        got = z.cpu().numpy()
        assert np.array_equal(got, ref)
        om = sketch_matrix(n, d, kind, seed, zeta)
        bound = np.asarray(abs(om) @ np.abs(xh)).ravel()
        assert np.all(np.abs(got - np.asarray(om @ xh).ravel()) <= 64 * U64 * bound + 1e-300)


def test_noalloc_sketch_rejects_sizes_beyond_the_scratch(lib, cuda):
    x = cuda.zeros(100, dtype=cuda.float64, device="cuda")
    z = cuda.zeros(2048, dtype=cuda.float64, device="cuda")
    for args in [(100, 1025, "sparse", 8), (100, 0, "sparse", 8), (0, 10, "sparse", 8), (100, 10, "sparse", 9),
                 (100, 4, "sparse", 5)]:
        with pytest.raises(P.RksError) as ei:
            P.rks_sketch_noalloc(*args, 1, x, z)
        assert ei.value.code == -1
        if args[1] == 1025:
            assert "1024" in P.rks_last_error(None)
    with pytest.raises(P.RksError):
        P.rks_sketch_noalloc(100, 10, "sparse", 8, 1, None, z)
