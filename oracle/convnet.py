"""Plain FP64 reference of the learned-start network (test infrastructure only).

The network maps the velocity field of a convection-diffusion operator,
sampled on a coarse h x w grid (2 channels), to one start vector on that grid.
Layers are 3x3 dilated convolutions with zero padding ("same" size), ReLU
after every layer but the last.  The loss of a prediction u against the
target invariant subspace V (orthonormal columns) is
    L(u) = 1 - ||V^T u||^2 / ||u||^2,
the fraction of u outside span(V), averaged over the batch; it does not
depend on the scale or sign of u, nor on the basis chosen for span(V).
Everything is written out with loops over the 9 taps; a reader can check
each formula against its definition.
"""
import numpy as np


def conv3x3(x, w, b, dil):
    """y[b,o,i,j] = bias[o] + sum_{c,di,dj} w[o,c,di,dj] x[b,c,i+dil(di-1),j+dil(dj-1)] (zero outside)."""
    B, C, H, W = x.shape
    O = w.shape[0]
    y = np.zeros((B, O, H, W))
    y += b[None, :, None, None]
    for di in range(3):
        for dj in range(3):
            oi, oj = dil * (di - 1), dil * (dj - 1)
            xs = np.zeros_like(x)
            i0, i1 = max(0, -oi), min(H, H - oi)
            j0, j1 = max(0, -oj), min(W, W - oj)
            xs[:, :, i0:i1, j0:j1] = x[:, :, i0 + oi:i1 + oi, j0 + oj:j1 + oj]
            y += np.einsum("oc,bcij->boij", w[:, :, di, dj], xs)
    return y


def conv3x3_backward(x, w, dy, dil):
    """Gradients of sum(dy * conv3x3(x, w, b, dil)) with respect to x, w, b."""
    B, C, H, W = x.shape
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    db = dy.sum(axis=(0, 2, 3))
    for di in range(3):
        for dj in range(3):
            oi, oj = dil * (di - 1), dil * (dj - 1)
            i0, i1 = max(0, -oi), min(H, H - oi)
            j0, j1 = max(0, -oj), min(W, W - oj)
            xs = np.zeros_like(x)
            xs[:, :, i0:i1, j0:j1] = x[:, :, i0 + oi:i1 + oi, j0 + oj:j1 + oj]
            dw[:, :, di, dj] = np.einsum("boij,bcij->oc", dy, xs)
            g = np.einsum("oc,boij->bcij", w[:, :, di, dj], dy)
            dx[:, :, i0 + oi:i1 + oi, j0 + oj:j1 + oj] += g[:, :, i0:i1, j0:j1]
    return dx, dw, db


def subspace_loss(u, V):
    """Mean over the batch of 1 - ||V_b^T u_b||^2/||u_b||^2 and its gradient.
    u: (B, P) predictions, V: (B, P, K) orthonormal target bases."""
    B = u.shape[0]
    p = np.einsum("bpk,bp->bk", V, u)
    uu = np.einsum("bp,bp->b", u, u)
    rho = np.einsum("bk,bk->b", p, p) / uu
    loss = np.mean(1.0 - rho)
    Vp = np.einsum("bpk,bk->bp", V, p)
    du = -2.0 * (Vp - rho[:, None] * u) / uu[:, None] / B
    return loss, du


class Net:
    """Dilated 3x3 convolution stack (plain NumPy)."""

    def __init__(self, params, dils):
        self.params = params   # list of (w, b)
        self.dils = dils

    def forward(self, x):
        acts = [x]
        h = x
        for li, ((w, b), d) in enumerate(zip(self.params, self.dils)):
            h = conv3x3(h, w, b, d)
            if li + 1 < len(self.params):
                h = np.maximum(h, 0.0)
            acts.append(h)
        return h, acts

    def backward(self, acts, dout):
        grads = [None] * len(self.params)
        g = dout
        for li in reversed(range(len(self.params))):
            w, b = self.params[li]
            if li + 1 < len(self.params):
                g = g * (acts[li + 1] > 0)
            dx, dw, db = conv3x3_backward(acts[li], w, g, self.dils[li])
            grads[li] = (dw, db)
            g = dx
        return grads


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def upsample_bilinear(u, H, W):
    """Bilinear resampling of u (h, w) to (H, W) with half-pixel centres:
    output pixel (I, J) samples input coordinates ((I+0.5) h/H - 0.5,
    (J+0.5) w/W - 0.5), clamped to the grid."""
    h, w = u.shape
    out = np.zeros((H, W))
    for I in range(H):
        y = min(max((I + 0.5) * h / H - 0.5, 0.0), h - 1.0)
        y0 = int(np.floor(y))
        y1 = min(y0 + 1, h - 1)
        fy = y - y0
        for J in range(W):
            x = min(max((J + 0.5) * w / W - 0.5, 0.0), w - 1.0)
            x0 = int(np.floor(x))
            x1 = min(x0 + 1, w - 1)
            fx = x - x0
            out[I, J] = ((1 - fy) * ((1 - fx) * u[y0, x0] + fx * u[y0, x1])
                         + fy * ((1 - fx) * u[y1, x0] + fx * u[y1, x1]))
    return out
