"""The GPU's final answer on the 100^2 convection-diffusion workload (the
small benchmark configuration: LR, k = 10, m = 40, Gaussian sketch d = 80,
seeds 0 / 1) against the closed-form spectrum.

The solve stops when every pair's FP64 residual is verified to be <= 1e-8.
It keeps k + (m - k)/4 Schur vectors per restart: with Algorithm 1's
truncation to k this strongly non-normal operator converges in about 130
restarts or stalls at the 300-restart cap depending on the rounding order of
the sums, while the larger restart size converges in about 34 either way.
First-order perturbation theory bounds each eigenvalue's error by
kappa(lambda) * ||A x - lambda x|| / ||x|| (kappa from the closed-form left
and right eigenvectors); the bar is twice that bound.  The wanted set is
unique because the gap between the 10th and 11th eigenvalue (9.64) exceeds
every bound.
"""
import numpy as np
import pytest

import paper_2508_05400_amd as P
from tests.closed_form import convdiff_eigs_kappa
from workloads import named_config

pytestmark = pytest.mark.gpu


def test_cd2d_100_against_closed_form(lib, cuda):
    cfg = named_config("cd2d-100")
    A = cfg["matrix"]()
    with P.Solver.from_csr(A, k=cfg["k"], m=cfg["m"], d=cfg["d"], which=cfg["which"], tol=cfg["tol"],
                           sketch_kind=cfg["sketch"], sketch_seed=cfg["sketch_seed"],
                           start_seed=cfg["start_seed"], resid_tol=1e-8, keep=-1) as s:
        code = s.solve()
        print(f"cd2d-100: code {code} restarts {s.stats.restarts} stop {s.stats.stop_reason}", flush=True)
        assert code == 0, P.rks_last_error(s.ctx)
        lam, X, res = s.eigpairs()
    import scipy.sparse as sp
    Sp = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    nA = abs(Sp).sum(axis=0).max()
    L, K = convdiff_eigs_kappa(100, (20.0, 10.0))
    order = np.argsort(-L)
    L, K = L[order], K[order]
    assert L[9] - L[10] > 9.0
    got = np.sort(lam.real)[::-1][:10]
    assert np.max(np.abs(lam.imag)) <= 1e-6 * L[0]
    assert res.max() <= 1e-8
    bound = 2.0 * K[:10] * res.max() * nA
    err = np.abs(got - L[:10])
    print("eigenvalue errors", err, "bounds", bound, flush=True)
    assert np.all(err <= bound), (err, bound)
