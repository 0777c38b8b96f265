"""Learned start vector for rKS on a parametric operator family.

The start vector u1 of Algorithm 1 is a free input (the paper draws it at
random, Section 2.1); restarting acts as a polynomial filter on it
(Section 3.2), so a start concentrated in the wanted invariant subspace can
save restarts.  This module trains a small network to propose it for the
2D convection-diffusion family with a random Fourier velocity field:

  features : the two velocity components averaged over 8x8 blocks -> 2x64x64
  network  : 3x3 convolutions, dilations 1,2,4,8,16,1, 16 channels, ReLU
             (receptive field covers the whole 64x64 grid)
  target   : the wanted invariant subspace computed by rKS itself, averaged
             over the same blocks and orthonormalised (64^2 x K)
  loss     : fraction of the prediction outside that subspace
  start    : the prediction resampled bilinearly to the full grid; the plain
             seeded random start remains the fallback

Every tensor operation of training and inference runs in the library's HIP
kernels (rks_net_*); torch only provides device memory.

  python -m paper_2508_05400_amd.learned_start --train 2000 --test 200 --out DIR
  python -m paper_2508_05400_amd.learned_start --eval-only --keep -1 --test 200 --out DIR
      (held-out comparison only, with the committed weights and a given restart size)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import _binding as B

LAYERS = [(2, 16, 1), (16, 16, 2), (16, 16, 4), (16, 16, 8), (16, 16, 16), (16, 1, 1)]  # (Cin, Cout, dilation)
GRID = 64
KPAD = 17  # wanted pairs k = 16, or 17 when a conjugate pair straddles the boundary
FAMILY = dict(N=512, k=16, m=48, d=192, which="SR", tol=1e-10, sketch="sparse", sketch_seed=5, start_seed=1)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_start_cd2d512.npz")


def block_mean(field: np.ndarray, N: int, g: int = GRID) -> np.ndarray:
    f = N // g
    return field.reshape(g, f, g, f).mean(axis=(1, 3))


def features(beta_x: np.ndarray, beta_y: np.ndarray, N: int) -> np.ndarray:
    """2 x 64 x 64 network input from the velocity field sampled at the grid nodes."""
    return np.stack([block_mean(beta_x.reshape(N, N), N), block_mean(beta_y.reshape(N, N), N)]) / 40.0


def target_basis(X: np.ndarray, N: int) -> np.ndarray:
    """Orthonormal basis (64^2 x KPAD, zero padded) of the block-averaged Ritz vectors."""
    cols = [block_mean(X[:, j].reshape(N, N), N).ravel() for j in range(X.shape[1])]
    Q, R = np.linalg.qr(np.stack(cols, axis=1))
    keep = np.abs(np.diag(R)) > 1e-12 * np.abs(np.diag(R)).max()
    Q = Q[:, keep]
    V = np.zeros((GRID * GRID, KPAD))
    V[:, :min(Q.shape[1], KPAD)] = Q[:, :KPAD]
    return V


class StartNet:
    """Parameters and Adam state on the device; passes through rks_net_* kernels."""

    def __init__(self, seed: int = 0):
        import torch
        self.torch = torch
        rng = np.random.default_rng(seed)
        self.w, self.b = [], []
        for cin, cout, _ in LAYERS:
            std = np.sqrt(2.0 / (cin * 9))
            self.w.append(torch.tensor(rng.standard_normal((cout, cin, 3, 3)) * std, dtype=torch.float32,
                                       device="cuda"))
            self.b.append(torch.zeros(cout, dtype=torch.float32, device="cuda"))
        self.m = [torch.zeros_like(p) for p in self.w + self.b]
        self.v = [torch.zeros_like(p) for p in self.w + self.b]
        self.t = 0

    def forward(self, x):
        """x: (Bn, 2, 64, 64) float32 device tensor -> list of activations."""
        torch = self.torch
        acts = [x.contiguous()]
        Bn = x.shape[0]
        for li, (cin, cout, dil) in enumerate(LAYERS):
            y = torch.empty((Bn, cout, GRID, GRID), dtype=torch.float32, device="cuda")
            B.rks_net_conv3x3_forward(acts[-1], self.w[li], self.b[li], y, Bn, cin, cout, GRID, GRID, dil,
                                      li + 1 < len(LAYERS))
            acts.append(y)
        return acts

    def backward(self, acts, dout):
        torch = self.torch
        Bn = acts[0].shape[0]
        gw, gb = [None] * len(LAYERS), [None] * len(LAYERS)
        g = dout.contiguous()
        for li in reversed(range(len(LAYERS))):
            cin, cout, dil = LAYERS[li]
            dw = torch.empty_like(self.w[li])
            db = torch.empty_like(self.b[li])
            dx = torch.empty_like(acts[li]) if li > 0 else None
            relu = li + 1 < len(LAYERS)
            B.rks_net_conv3x3_backward(acts[li], self.w[li], acts[li + 1] if relu else None, g, dx, dw, db, Bn,
                                       cin, cout, GRID, GRID, dil, relu)
            gw[li], gb[li] = dw, db
            g = dx
        return gw, gb

    def loss_and_grad(self, out, V):
        torch = self.torch
        Bn = out.shape[0]
        loss = torch.empty(Bn, dtype=torch.float32, device="cuda")
        du = torch.empty((Bn, GRID * GRID), dtype=torch.float32, device="cuda")
        B.rks_net_subspace_loss(out.reshape(Bn, GRID * GRID), V, loss, du, Bn, GRID * GRID, V.shape[2])
        return loss, du.reshape(out.shape)

    def adam(self, gw, gb, lr):
        self.t += 1
        for p, g, m, v in zip(self.w + self.b, gw + gb, self.m, self.v):
            B.rks_net_adam(p, g, m, v, p.numel(), lr, self.t)

    def predict(self, feats: np.ndarray):
        torch = self.torch
        x = torch.tensor(feats[None], dtype=torch.float32, device="cuda")
        return self.forward(x)[-1]

    def start_vector(self, feats: np.ndarray, N: int):
        """FP64 device start vector on the full N x N grid."""
        torch = self.torch
        u = self.predict(feats)
        out = torch.empty(N * N, dtype=torch.float64, device="cuda")
        B.rks_net_upsample(u, GRID, GRID, out, N, N)
        return out

    def save(self, path: str, meta: dict):
        arrs = {f"w{i}": w.cpu().numpy() for i, w in enumerate(self.w)}
        arrs.update({f"b{i}": b.cpu().numpy() for i, b in enumerate(self.b)})
        np.savez(path, meta=json.dumps(meta), **arrs)

    @classmethod
    def load(cls, path: str):
        import torch
        net = cls(seed=0)
        with np.load(path, allow_pickle=False) as z:
            for i in range(len(LAYERS)):
                net.w[i] = torch.tensor(z[f"w{i}"], dtype=torch.float32, device="cuda")
                net.b[i] = torch.tensor(z[f"b{i}"], dtype=torch.float32, device="cuda")
        return net


def start_for(feats: np.ndarray, N: int, weights: str = WEIGHTS, net=None):
    """Start vector for rks_solve: the network's proposal as an FP64 device
    vector, or None (the solver's own seeded random start) when no trained
    weights exist or the proposal is not a usable vector (non-finite or zero)."""
    if net is None:
        if not os.path.exists(weights):
            return None
        net = StartNet.load(weights)
    u = net.start_vector(feats, N)
    nrm = float(u.norm())
    if not np.isfinite(nrm) or nrm == 0.0:
        return None
    return u


def instance(i: int):
    """Operator i of the family (seed 10000 + i) and its velocity field."""
    from workloads import convdiff2d_field, fourier_beta_field
    N = FAMILY["N"]
    A = convdiff2d_field(N, 10000 + i)
    bx, by = fourier_beta_field(N, 10000 + i)
    return A, features(bx, by, N)


def solve(A, u0=None, resid_tol=1e-5, want_vectors=True, keep=0):
    """rKS on one family member to a verified residual; returns (stats, Ritz vectors, seconds).
    The Ritz vectors at exit are returned even when the restart cap is hit.
    keep is the restart size (0: k, as in Algorithm 1; -1: automatic)."""
    import torch
    from . import Solver
    f = FAMILY
    with Solver.from_csr(A, k=f["k"], m=f["m"], d=f["d"], which=f["which"], tol=f["tol"], sketch_kind=f["sketch"],
                         sketch_seed=f["sketch_seed"], start_seed=f["start_seed"], resid_tol=resid_tol,
                         keep=keep) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code = s.solve(u0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = s.stats.as_dict()
        st["code"] = code
        _, X, res = s.eigpairs(want_vectors=want_vectors, want_resid=True)
        st["max_resid_final"] = float(res.max())
    return st, X, dt


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--target", type=float, default=1e-5, help="verified residual of the comparison")
    ap.add_argument("--final", type=int, default=50, help="test instances also run to residual 1e-8")
    ap.add_argument("--out", default="learned_out")
    ap.add_argument("--weights", default=None)
    ap.add_argument("--keep", type=int, default=0, help="restart size of every solve (0: k, -1: automatic)")
    ap.add_argument("--eval-only", action="store_true",
                    help="skip data generation and training: compare the weights (default: the committed ones) "
                         "with the random start on the held-out instances")
    args = ap.parse_args(argv)
    if args.eval_only:
        return evaluate(args)
    import torch
    os.makedirs(args.out, exist_ok=True)
    N = FAMILY["N"]
    t_start = time.time()

    def log(msg):
        print(f"[{time.time() - t_start:7.1f}s] {msg}", flush=True)

    # 1. data: rKS with the plain random start on every instance; the Ritz
    #    subspace at exit is the training target (converged or not)
    feats, targets, base = [], [], []
    ntot = args.train + args.test
    seeds = list(range(args.train)) + [100000 + j for j in range(args.test)]
    for i, sd in enumerate(seeds):
        A, f = instance(sd)
        st, X, dt = solve(A, resid_tol=args.target, keep=args.keep)
        base.append({"seed": 10000 + sd, "restarts": st["restarts"], "matvecs": st["matvecs"], "time_s": dt,
                     "code": st["code"], "resid": st["max_resid_final"]})
        feats.append(f)
        targets.append(target_basis(X, N))
        if (i + 1) % 25 == 0 or i + 1 == ntot:
            log(f"data {i + 1}/{ntot}: last {dt:.3f}s restarts={st['restarts']} code={st['code']}")
    X_tr = torch.tensor(np.stack(feats[:args.train]), dtype=torch.float32, device="cuda")
    V_tr = torch.tensor(np.stack(targets[:args.train]), dtype=torch.float32, device="cuda")
    net = StartNet(seed=0)
    rng = np.random.default_rng(1)
    hist = []
    for ep in range(args.epochs):
        perm = rng.permutation(args.train)
        tot = 0.0
        for s0 in range(0, len(perm), args.batch):
            sel = torch.tensor(perm[s0:s0 + args.batch], device="cuda")
            acts = net.forward(X_tr[sel])
            loss, du = net.loss_and_grad(acts[-1], V_tr[sel])
            gw, gb = net.backward(acts, du)
            net.adam(gw, gb, args.lr)
            tot += float(loss.sum())
        hist.append(tot / len(perm))
        if (ep + 1) % 5 == 0 or ep == 0:
            log(f"epoch {ep + 1}/{args.epochs}: mean training loss {hist[-1]:.4f}")
    wpath = args.weights or os.path.join(args.out, "learned_start_cd2d512.npz")
    net.save(wpath, {"layers": LAYERS, "family": FAMILY, "train": args.train, "epochs": args.epochs,
                     "loss_history": hist})
    # 2. held-out instances: learned start vs the random start
    evals = []
    for j in range(args.test):
        i = args.train + j
        A, f = instance(seeds[i])
        u0 = net.start_vector(f, N)
        st, _, dt = solve(A, u0, resid_tol=args.target, want_vectors=False, keep=args.keep)
        Vt = torch.tensor(targets[i][None], dtype=torch.float32, device="cuda")
        l, _ = net.loss_and_grad(net.predict(f), Vt)
        e = {"seed": base[i]["seed"], "random_restarts": base[i]["restarts"], "random_matvecs": base[i]["matvecs"],
             "random_time_s": base[i]["time_s"], "random_code": base[i]["code"],
             "learned_restarts": st["restarts"], "learned_matvecs": st["matvecs"], "learned_time_s": dt,
             "learned_code": st["code"], "subspace_fraction": 1.0 - float(l[0])}
        if j < args.final:
            sr, _, tr = solve(A, None, resid_tol=1e-8, want_vectors=False, keep=args.keep)
            sl, _, tl = solve(A, u0, resid_tol=1e-8, want_vectors=False, keep=args.keep)
            e.update({"random_1e-8_code": sr["code"], "random_1e-8_restarts": sr["restarts"],
                      "random_1e-8_time_s": tr, "learned_1e-8_code": sl["code"],
                      "learned_1e-8_restarts": sl["restarts"], "learned_1e-8_time_s": tl})
        evals.append(e)
        if (j + 1) % 25 == 0:
            log(f"eval {j + 1}/{args.test}")
    rm = np.array([e["random_matvecs"] for e in evals], dtype=float)
    lm = np.array([e["learned_matvecs"] for e in evals], dtype=float)
    rt = np.array([e["random_time_s"] for e in evals])
    lt = np.array([e["learned_time_s"] for e in evals])
    fin = [e for e in evals if "random_1e-8_code" in e]
    summary = {"train": args.train, "test": len(evals), "epochs": args.epochs, "target_resid": args.target,
               "final_training_loss": hist[-1],
               "mean_subspace_fraction_learned": float(np.mean([e["subspace_fraction"] for e in evals])),
               "mean_subspace_fraction_random": float(KPAD / (GRID * GRID)),
               "median_matvec_ratio_learned_over_random": float(np.median(lm / rm)),
               "mean_matvecs_random": float(rm.mean()), "mean_matvecs_learned": float(lm.mean()),
               "mean_time_random_s": float(rt.mean()), "mean_time_learned_s": float(lt.mean()),
               "reached_target_random": int(sum(e["random_code"] == 0 for e in evals)),
               "reached_target_learned": int(sum(e["learned_code"] == 0 for e in evals)),
               "final_1e-8_instances": len(fin),
               "reached_1e-8_random": int(sum(e["random_1e-8_code"] == 0 for e in fin)),
               "reached_1e-8_learned": int(sum(e["learned_1e-8_code"] == 0 for e in fin))}
    with open(os.path.join(args.out, "learned_start_results.json"), "w") as fh:
        json.dump({"summary": summary, "loss_history": hist, "eval": evals, "data": base}, fh)
    log("summary " + json.dumps(summary))
    return summary


def evaluate(args):
    """Held-out comparison with trained weights: for each test instance the
    random start and the network's start, both to the verified residual
    args.target, and the first args.final instances also to 1e-8."""
    N = FAMILY["N"]
    t_start = time.time()
    net = StartNet.load(args.weights or WEIGHTS)
    evals = []
    for j in range(args.test):
        A, f = instance(100000 + j)
        u0 = net.start_vector(f, N)
        sr, Xr, tr = solve(A, None, resid_tol=args.target, want_vectors=True, keep=args.keep)
        sl, _, tl = solve(A, u0, resid_tol=args.target, want_vectors=False, keep=args.keep)
        import torch
        Vt = torch.tensor(target_basis(Xr, N)[None], dtype=torch.float32, device="cuda")
        l, _ = net.loss_and_grad(net.predict(f), Vt)
        e = {"seed": 110000 + j, "random_restarts": sr["restarts"], "random_matvecs": sr["matvecs"],
             "random_time_s": tr, "random_code": sr["code"], "learned_restarts": sl["restarts"],
             "learned_matvecs": sl["matvecs"], "learned_time_s": tl, "learned_code": sl["code"],
             "subspace_fraction": 1.0 - float(l[0])}
        if j < args.final:
            s8r, _, t8r = solve(A, None, resid_tol=1e-8, want_vectors=False, keep=args.keep)
            s8l, _, t8l = solve(A, u0, resid_tol=1e-8, want_vectors=False, keep=args.keep)
            e.update({"random_1e-8_code": s8r["code"], "random_1e-8_restarts": s8r["restarts"],
                      "random_1e-8_matvecs": s8r["matvecs"], "random_1e-8_time_s": t8r,
                      "learned_1e-8_code": s8l["code"], "learned_1e-8_restarts": s8l["restarts"],
                      "learned_1e-8_matvecs": s8l["matvecs"], "learned_1e-8_time_s": t8l})
        evals.append(e)
        if (j + 1) % 10 == 0:
            print(f"[{time.time() - t_start:7.1f}s] eval {j + 1}/{args.test}", flush=True)
    rm = np.array([e["random_matvecs"] for e in evals], dtype=float)
    lm = np.array([e["learned_matvecs"] for e in evals], dtype=float)
    both = [e for e in evals if e["random_code"] == 0 and e["learned_code"] == 0]
    fin = [e for e in evals if "random_1e-8_code" in e]
    fin_both = [e for e in fin if e["random_1e-8_code"] == 0 and e["learned_1e-8_code"] == 0]
    summary = {"test": len(evals), "keep": args.keep, "target_resid": args.target,
               "mean_subspace_fraction_learned": float(np.mean([e["subspace_fraction"] for e in evals])),
               "median_matvec_ratio_learned_over_random": float(np.median(lm / rm)),
               "mean_matvecs_random": float(rm.mean()), "mean_matvecs_learned": float(lm.mean()),
               "mean_time_random_s": float(np.mean([e["random_time_s"] for e in evals])),
               "mean_time_learned_s": float(np.mean([e["learned_time_s"] for e in evals])),
               "reached_target_random": int(sum(e["random_code"] == 0 for e in evals)),
               "reached_target_learned": int(sum(e["learned_code"] == 0 for e in evals)),
               "median_matvec_ratio_where_both_reached": (float(np.median(
                   [e["learned_matvecs"] / e["random_matvecs"] for e in both])) if both else None),
               "final_1e-8_instances": len(fin),
               "reached_1e-8_random": int(sum(e["random_1e-8_code"] == 0 for e in fin)),
               "reached_1e-8_learned": int(sum(e["learned_1e-8_code"] == 0 for e in fin)),
               "median_1e-8_matvec_ratio_where_both_reached": (float(np.median(
                   [e["learned_1e-8_matvecs"] / e["random_1e-8_matvecs"] for e in fin_both])) if fin_both else None),
               "mean_1e-8_time_random_s": (float(np.mean([e["random_1e-8_time_s"] for e in fin])) if fin else None),
               "mean_1e-8_time_learned_s": (float(np.mean([e["learned_1e-8_time_s"] for e in fin])) if fin else None)}
    os.makedirs(args.out, exist_ok=True)
    what = (f"held-out evaluation of {os.path.basename(args.weights or WEIGHTS)}: {len(evals)} instances (seeds "
            f"110000..{110000 + len(evals) - 1}) of the 512^2 variable-velocity convection-diffusion family, rKS "
            f"k=16 m=48 d=192 SR sparse-sign seed 5, restart size keep={args.keep} (0: k, -1: k + (m-k)/4), "
            f"random start against the network's start, verified residual {args.target:g} (and 1e-8 on the "
            f"first {len(fin)}); code 0 = reached, 1 = restart cap 300")
    command = (f"python -m paper_2508_05400_amd.learned_start --eval-only --keep {args.keep} --test {args.test} "
               f"--final {args.final} --target {args.target:g} --out <dir>")
    with open(os.path.join(args.out, "learned_start_eval.json"), "w") as fh:
        json.dump({"what": what, "command": command, "summary": summary, "eval": evals}, fh, indent=0)
    print("summary " + json.dumps(summary), flush=True)
    return summary


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
