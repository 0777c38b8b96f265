"""Pins of the learned-start network oracle (plain FP64 NumPy)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle.convnet import Net, adam_step, conv3x3, conv3x3_backward, subspace_loss, upsample_bilinear


def _dilated_kernel(k, d):
    kd = np.zeros((2 * d + 1, 2 * d + 1))
    kd[::d, ::d] = k
    return kd


@pytest.mark.parametrize("dil", [1, 2, 5])
def test_conv_matches_library_correlation(dil):
    rng = np.random.default_rng(dil)
    x = rng.standard_normal((2, 3, 12, 10))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = conv3x3(x, w, b, dil)
    for bb in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[bb, c], _dilated_kernel(w[o, c], dil), mode="same", boundary="fill")
                             for c in range(3))
            assert np.allclose(y[bb, o], ref, atol=1e-12)


def _fd(f, x, eps=1e-6):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = x[i]
        x[i] = old + eps
        fp = f()
        x[i] = old - eps
        fm = f()
        x[i] = old
        g[i] = (fp - fm) / (2 * eps)
    return g


@pytest.mark.parametrize("dil", [1, 3])
def test_conv_backward_finite_differences(dil):
    rng = np.random.default_rng(10 + dil)
    x = rng.standard_normal((2, 2, 7, 6))
    w = rng.standard_normal((3, 2, 3, 3))
    b = rng.standard_normal(3)
    dy = rng.standard_normal((2, 3, 7, 6))
    f = lambda: float(np.sum(dy * conv3x3(x, w, b, dil)))
    dx, dw, db = conv3x3_backward(x, w, dy, dil)
    assert np.allclose(dx, _fd(f, x), atol=1e-6)
    assert np.allclose(dw, _fd(f, w), atol=1e-6)
    assert np.allclose(db, _fd(f, b), atol=1e-6)


def test_subspace_loss_closed_forms_and_gradient():
    rng = np.random.default_rng(3)
    P, K = 50, 4
    V, _ = np.linalg.qr(rng.standard_normal((P, K)))
    inside = V @ rng.standard_normal(K)
    outside = rng.standard_normal(P)
    outside -= V @ (V.T @ outside)
    l_in, _ = subspace_loss(inside[None], V[None])
    l_out, _ = subspace_loss(outside[None], V[None])
    assert abs(l_in) < 1e-14 and abs(l_out - 1.0) < 1e-14
    u = rng.standard_normal((3, P))
    Vb = np.stack([V, np.linalg.qr(rng.standard_normal((P, K)))[0], V])
    l1, g = subspace_loss(u, Vb)
    # invariance: scaling u, rotating the basis of span(V)
    Qk, _ = np.linalg.qr(rng.standard_normal((K, K)))
    l2, _ = subspace_loss(-3.0 * u, Vb @ Qk)
    assert abs(l1 - l2) < 1e-13
    f = lambda: float(subspace_loss(u, Vb)[0])
    assert np.allclose(g, _fd(f, u), atol=1e-7)


def test_network_backward_finite_differences():
    rng = np.random.default_rng(5)
    dils = [1, 2, 1]
    shapes = [(4, 2), (4, 4), (1, 4)]
    params = [(0.3 * rng.standard_normal((o, c, 3, 3)), 0.1 * rng.standard_normal(o)) for o, c in shapes]
    net = Net(params, dils)
    x = rng.standard_normal((2, 2, 8, 8))
    V = np.stack([np.linalg.qr(rng.standard_normal((64, 3)))[0] for _ in range(2)])

    def loss():
        out, _ = net.forward(x)
        return float(subspace_loss(out.reshape(2, 64), V)[0])

    out, acts = net.forward(x)
    _, du = subspace_loss(out.reshape(2, 64), V)
    grads = net.backward(acts, du.reshape(out.shape))
    for (w, b), (dw, db) in zip(params, grads):
        assert np.allclose(dw, _fd(loss, w), atol=1e-6, rtol=1e-4)
        assert np.allclose(db, _fd(loss, b), atol=1e-6, rtol=1e-4)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    w = np.zeros(3)
    w1, m, v = adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(w1, -0.01 * g / (np.abs(g) + 1e-8))


def test_upsample_bilinear_separable_interp():
    """Bilinear resampling equals 1D linear interpolation along each axis."""
    rng = np.random.default_rng(7)
    u = rng.standard_normal((5, 7))
    H, W = 20, 14
    out = upsample_bilinear(u, H, W)
    ys = np.clip((np.arange(H) + 0.5) * 5 / H - 0.5, 0, 4)
    xs = np.clip((np.arange(W) + 0.5) * 7 / W - 0.5, 0, 6)
    rows = np.stack([np.interp(xs, np.arange(7), u[i]) for i in range(5)])
    ref = np.stack([np.interp(ys, np.arange(5), rows[:, j]) for j in range(W)], axis=1)
    assert np.allclose(out, ref, atol=1e-13)
    assert np.allclose(upsample_bilinear(np.full((3, 3), 2.5), 12, 12), 2.5)
