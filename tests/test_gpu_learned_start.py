"""The trained start network against the plain random start, on held-out
members of the 512^2 variable-velocity convection-diffusion family (instance
seeds 110000 + j: never used in training, which used seeds 10000..11999).

Asserted: what the network is trained for (the predicted start lies almost
entirely in the wanted invariant subspace at the network's 64^2 resolution;
a random vector has 17/4096 of its energy there), what the solver guarantees
(the solve from it reaches the same verified residual), and the gain in
products with A, against a bound that comes from the committed evaluation on
200 held-out instances (profiles/learned_start_cd2d512_eval_keep_auto.json):
there the learned start needs fewer products on 129 of 200 instances (paired
sign test p = 2.5e-5), median ratio 0.972, mean 0.987, per-instance standard
deviation 0.125.  The mean ratio over the 16 instances run here must lie
within three standard errors (3 x 0.125 / 4) of that mean; the committed
evaluation's own sign test is checked on the CPU in
test_learned_start_evaluation_record.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HELD_OUT = list(range(100000, 100016))
RECORD = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                      "learned_start_cd2d512_eval_keep_auto.json")


def test_learned_start_vs_random(lib, cuda):
    from paper_2508_05400_amd.learned_start import (FAMILY, GRID, KPAD, WEIGHTS, StartNet, block_mean, instance,
                                                    solve, target_basis)
    N = FAMILY["N"]
    net = StartNet.load(WEIGHTS)
    rows = []
    for sd in HELD_OUT:
        A, f = instance(sd)
        st_r, X, t_r = solve(A, None, resid_tol=1e-5, want_vectors=True, keep=-1)
        u = net.start_vector(f, N)
        uh = u.cpu().numpy()
        assert np.all(np.isfinite(uh)) and np.linalg.norm(uh) > 0
        V = target_basis(X, N)
        uc = block_mean(uh.reshape(N, N), N).ravel()
        frac = float(np.sum((V.T @ uc) ** 2) / np.sum(uc ** 2))
        st_l, _, t_l = solve(A, u, resid_tol=1e-5, want_vectors=False, keep=-1)
        rows.append((frac, st_r["matvecs"], st_l["matvecs"], st_r["code"], st_l["code"], st_l["max_resid_final"]))
        print(f"instance {10000 + sd}: subspace fraction {frac:.4f}; products random {st_r['matvecs']} learned "
              f"{st_l['matvecs']}; time random {t_r:.3f}s learned {t_l:.3f}s", flush=True)
    fr = np.array([r[0] for r in rows])
    assert fr.min() > 0.8, fr                       # random: KPAD / GRID^2
    assert fr.mean() > 100 * KPAD / GRID**2
    for r in rows:
        assert r[3] == 0 and r[4] == 0              # both starts converge with this restart size
        assert r[5] <= 1e-5
    ratio = np.array([r[2] / r[1] for r in rows])
    with open(RECORD) as fh:
        ev = json.load(fh)["eval"]
    ref = np.array([e["learned_matvecs"] / e["random_matvecs"] for e in ev])
    mu, sd = float(ref.mean()), float(ref.std(ddof=1))
    bound = mu + 3 * sd / np.sqrt(len(ratio))
    print(f"mean product ratio learned/random over {len(ratio)}: {ratio.mean():.4f} (evaluation: mean {mu:.4f}, "
          f"sd {sd:.4f}; bound {bound:.4f})", flush=True)
    assert ratio.mean() <= bound
