"""Per-kernel timing of the solver (rks_opts.profile): the events attached to
the launches must leave the numerics untouched and give durations that fit
inside the whole-step figure, for the sparse-sign sketch in both SpMV layouts
and for the Gaussian sketch (whose launchers run two kernels under one event
pair)."""
import numpy as np
import pytest

import paper_2508_05400_amd as P
from workloads import convdiff2d

pytestmark = pytest.mark.gpu


def _solve(A, profile, **kw):
    with P.Solver.from_csr(A, k=6, m=24, d=60, which="SR", tol=1e-10, sketch_seed=2, start_seed=1,
                           resid_tol=1e-8, max_restarts=40, keep=-1, profile=profile, **kw) as s:
        rc = s.solve()
        assert rc in (0, 1), P.rks_last_error(s.ctx)
        lam, _, _ = s.eigpairs(want_vectors=False, want_resid=False)
        return lam, s.stats.as_dict()


@pytest.mark.parametrize("kw", [dict(sketch_kind="sparse", spmv_layout="rows"),
                                dict(sketch_kind="sparse", spmv_layout="column_blocks"),
                                dict(sketch_kind="gauss")], ids=["sparse-rows", "sparse-cb", "gauss"])
def test_timing_leaves_results_unchanged_and_fits_the_step(lib, cuda, kw):
    A = convdiff2d(300, (50.0, 30.0))
    lam0, st0 = _solve(A, 0, **kw)
    lam1, st1 = _solve(A, 1, **kw)
    # the same solve to the last bit, with or without the events
    assert st1["restarts"] == st0["restarts"] and st1["matvecs"] == st0["matvecs"]
    assert np.array_equal(lam0, lam1)
    assert st0["n_timed_steps"] == 0 and st0["t_update"] == 0.0
    # profile = 1: every step is timed, alternately per kernel and as a whole
    ns, nw = st1["n_timed_steps"], st1["n_timed_whole"]
    assert ns > 0 and nw > 0 and abs(ns - nw) <= 1
    assert ns + nw == st1["n_update"]
    per = [st1[k] / ns for k in ("t_spmv", "t_reduce", "t_update")]
    assert all(p > 0.0 for p in per), per
    assert st1["t_ls"] == 0.0  # the least squares runs inside the update launch
    whole = st1["t_step"] / nw
    # the three kernels lie inside the step, which adds launch gaps and its event pair (the two
    # samples are alternate steps, whose column counts differ by one)
    assert sum(per) <= whole * 1.10, (per, whole)
    assert sum(per) >= 0.3 * whole, (per, whole)
    assert st1["n_timed_rotate"] == st1["n_rotate"] > 0 and st1["t_rotate"] > 0.0
