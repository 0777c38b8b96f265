"""GPU parity of the learned-start network kernels against the FP64 NumPy
oracle (oracle/convnet.py), and the trained network's effect on rKS.

FP32 kernels: each output is a sum of at most 16*9 = 144 products (forward,
input gradient) or B*64*64 products (filter gradient); the bar is
rtol 2e-5 / atol 2e-5 * max|reference| for the former and 1e-4 for the
latter (FP32 unit roundoff 6e-8 times the summation length, with margin).
"""
import os

import numpy as np
import pytest

import paper_2508_05400_amd as P
from oracle.convnet import Net, adam_step, conv3x3, conv3x3_backward, subspace_loss, upsample_bilinear

pytestmark = pytest.mark.gpu


def t32(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("B,C,O,H,W,dil,relu", [(2, 2, 16, 64, 64, 1, 1), (3, 16, 16, 64, 64, 8, 1),
                                                  (1, 16, 1, 64, 64, 1, 0), (2, 5, 3, 13, 9, 2, 1)])
def test_conv_forward_backward(lib, cuda, B, C, O, H, W, dil, relu):
    torch = cuda
    rng = np.random.default_rng(B * 100 + C + dil)
    x = rng.standard_normal((B, C, H, W)).astype(np.float32)
    w = (0.3 * rng.standard_normal((O, C, 3, 3))).astype(np.float32)
    b = (0.1 * rng.standard_normal(O)).astype(np.float32)
    dy = rng.standard_normal((B, O, H, W)).astype(np.float32)
    xd, wd, bd, dyd = t32(torch, x), t32(torch, w), t32(torch, b), t32(torch, dy)
    y = torch.empty((B, O, H, W), dtype=torch.float32, device="cuda")
    P.rks_net_conv3x3_forward(xd, wd, bd, y, B, C, O, H, W, dil, relu)
    ref = conv3x3(x.astype(np.float64), w.astype(np.float64), b.astype(np.float64), dil)
    if relu:
        ref = np.maximum(ref, 0.0)
    scale = np.abs(ref).max()
    assert np.allclose(y.cpu().numpy(), ref, rtol=2e-5, atol=2e-5 * scale)
    dx = torch.empty_like(xd)
    dw = torch.empty_like(wd)
    db = torch.empty_like(bd)
    P.rks_net_conv3x3_backward(xd, wd, y if relu else None, dyd, dx, dw, db, B, C, O, H, W, dil, relu)
    g = dy.astype(np.float64) * ((ref > 0) if relu else 1.0)
    rdx, rdw, rdb = conv3x3_backward(x.astype(np.float64), w.astype(np.float64), g, dil)
    assert np.allclose(dx.cpu().numpy(), rdx, rtol=2e-5, atol=2e-5 * np.abs(rdx).max())
    assert np.allclose(dw.cpu().numpy(), rdw, rtol=1e-4, atol=1e-4 * np.abs(rdw).max())
    assert np.allclose(db.cpu().numpy(), rdb, rtol=1e-4, atol=1e-4 * np.abs(rdb).max())


def test_loss_adam_upsample(lib, cuda):
    torch = cuda
    rng = np.random.default_rng(3)
    Bn, Pp, K = 4, 4096, 17
    u = rng.standard_normal((Bn, Pp)).astype(np.float32)
    V = np.stack([np.linalg.qr(rng.standard_normal((Pp, K)))[0] for _ in range(Bn)])
    V[1, :, 16] = 0.0  # a padded column
    loss = torch.empty(Bn, dtype=torch.float32, device="cuda")
    du = torch.empty((Bn, Pp), dtype=torch.float32, device="cuda")
    P.rks_net_subspace_loss(t32(torch, u), t32(torch, V), loss, du, Bn, Pp, K)
    rl, rdu = subspace_loss(u.astype(np.float64), V)
    assert abs(float(loss.mean()) - rl) < 1e-5
    assert np.allclose(du.cpu().numpy(), rdu, rtol=1e-4, atol=1e-4 * np.abs(rdu).max())
    # Adam: three steps against the FP64 reference
    w0 = rng.standard_normal(1000).astype(np.float32)
    wd, md, vd = t32(torch, w0), torch.zeros(1000, device="cuda"), torch.zeros(1000, device="cuda")
    rw, rm, rv = w0.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for t in range(1, 4):
        g = rng.standard_normal(1000).astype(np.float32)
        P.rks_net_adam(wd, t32(torch, g), md, vd, 1000, 1e-2, t)
        rw, rm, rv = adam_step(rw, g.astype(np.float64), rm, rv, t, 1e-2)
    assert np.allclose(wd.cpu().numpy(), rw, atol=1e-5)
    # upsample 64x64 -> 512x512 (FP64 output)
    uu = rng.standard_normal((64, 64)).astype(np.float32)
    out = torch.empty(512 * 512, dtype=torch.float64, device="cuda")
    P.rks_net_upsample(t32(torch, uu), 64, 64, out, 512, 512)
    ref = upsample_bilinear(uu.astype(np.float64), 512, 512)
    assert np.allclose(out.cpu().numpy().reshape(512, 512), ref, atol=1e-12)


def test_network_gradient_matches_oracle(lib, cuda):
    """Full forward + loss + backward of the start network against the FP64 oracle."""
    from paper_2508_05400_amd.learned_start import LAYERS, StartNet
    torch = cuda
    net = StartNet(seed=3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 2, 64, 64)).astype(np.float32)
    V = np.stack([np.linalg.qr(rng.standard_normal((4096, 17)))[0] for _ in range(2)]).astype(np.float32)
    acts = net.forward(t32(torch, x))
    loss, du = net.loss_and_grad(acts[-1], t32(torch, V))
    gw, gb = net.backward(acts, du)
    params = [(w.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64))
              for w, b in zip(net.w, net.b)]
    ref = Net(params, [d for _, _, d in LAYERS])
    out, racts = ref.forward(x.astype(np.float64))
    rl, rdu = subspace_loss(out.reshape(2, -1), V.astype(np.float64))
    rgrads = ref.backward(racts, rdu.reshape(out.shape))
    assert abs(float(loss.mean()) - rl) < 1e-4
    for li in range(len(LAYERS)):
        rdw, rdb = rgrads[li]
        assert np.allclose(gw[li].cpu().numpy(), rdw, rtol=1e-3, atol=1e-3 * np.abs(rdw).max()), li
        assert np.allclose(gb[li].cpu().numpy(), rdb, rtol=1e-3, atol=1e-3 * np.abs(rdb).max()), li
