"""FP64 reference of the learned smoother's network (test infrastructure only).

The learned smoother is not in the paper: it is one of the build's required
extensions of the multigrid cycle (the smoothers of Algorithm 2).  Network on
one level's index grid (rows = y index j, columns = x index i):

    y = C3(relu(C2(relu(C1(z)))))

with C1: 1 -> 16, C2: 16 -> 16, C3: 16 -> 1 channels, 3x3 cross-correlation
with zero "same" padding, no biases (so the map is positively homogeneous).
Activations outside the domain mask are zero (padding at the domain boundary).

Precision model of the device implementation, reproduced here where it rounds:
weights are BF16 values; the first layer's activations are rounded to BF16
(round to nearest even) before the second layer, which multiplies BF16 operands
with FP32 accumulation; in the backward pass the second layer's output gradient
is rounded to BF16 before its two products.  `bf16_points=False` evaluates the
same network without those roundings (used to pin the gradients by finite
differences).

Loss: mean over the loss pixels of (y - t)^2.
"""
import numpy as np

TAPS = [(dy, dx) for dy in range(3) for dx in range(3)]


def bf16_round(a):
    """Round float64 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_weights(rng, channels=16):
    """He-style random weights (shapes [c_out, c_in, 3, 3])."""
    def w(co, ci):
        return rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci))
    return [w(channels, 1), w(channels, channels), w(1, channels) * 0.1]


def conv3x3(x, W):
    """y[co, j, i] = sum_ci sum_{dy,dx} W[co, ci, dy, dx] x[ci, j+dy-1, i+dx-1] (zero outside)."""
    ci, H, Wd = x.shape
    xp = np.zeros((ci, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((W.shape[0], H, Wd))
    for dy, dx in TAPS:
        y += np.einsum("oc,chw->ohw", W[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + Wd])
    return y


def conv3x3_transpose(g, W):
    """Adjoint of conv3x3 with respect to its input."""
    co, H, Wd = g.shape
    gp = np.zeros((co, H + 2, Wd + 2))
    gp[:, 1:-1, 1:-1] = g
    x = np.zeros((W.shape[1], H, Wd))
    for dy, dx in TAPS:
        # y[o, j, i] uses x[c, j+dy-1, i+dx-1]: x[c, a, b] receives g[o, a-dy+1, b-dx+1]
        x += np.einsum("oc,ohw->chw", W[:, :, dy, dx], gp[:, 2 - dy:2 - dy + H, 2 - dx:2 - dx + Wd])
    return x


def conv3x3_weight_grad(x, g):
    """dL/dW[co, ci, dy, dx] = sum_{j,i} g[co, j, i] x[ci, j+dy-1, i+dx-1]."""
    ci, H, Wd = x.shape
    xp = np.zeros((ci, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dW = np.zeros((g.shape[0], ci, 3, 3))
    for dy, dx in TAPS:
        dW[:, :, dy, dx] = np.einsum("ohw,chw->oc", g, xp[:, dy:dy + H, dx:dx + Wd])
    return dW


def forward(z, Ws, mask=None, bf16_points=True):
    """z: (H, W) input, mask: (H, W) domain indicator.  Returns (y, cache)."""
    z = np.asarray(z, dtype=np.float64)
    m = np.ones_like(z) if mask is None else np.asarray(mask, dtype=np.float64)
    W1, W2, W3 = Ws
    a1 = conv3x3(z[None], W1)
    h1 = np.maximum(a1, 0.0) * m
    h1q = bf16_round(h1) if bf16_points else h1
    a2 = conv3x3(h1q, W2)
    h2 = np.maximum(a2, 0.0) * m
    y = conv3x3(h2, W3)[0]
    return y, (z, m, a1, h1q, a2, h2)


def loss_and_grads(z, t, Ws, mask=None, loss_mask=None, bf16_points=True):
    """Loss = mean over loss pixels of (y - t)^2 and its gradients w.r.t. W1, W2, W3."""
    y, (z, m, a1, h1q, a2, h2) = forward(z, Ws, mask, bf16_points)
    lm = np.ones_like(y) if loss_mask is None else np.asarray(loss_mask, dtype=np.float64)
    cnt = lm.sum()
    d = (y - t) * lm
    loss = float(np.sum(d * d) / cnt)
    gy = 2.0 * d / cnt
    W1, W2, W3 = Ws
    dW3 = conv3x3_weight_grad(h2, gy[None])
    gh2 = conv3x3_transpose(gy[None], W3) * (a2 > 0) * m
    gh2q = bf16_round(gh2) if bf16_points else gh2
    dW2 = conv3x3_weight_grad(h1q, gh2q)
    gh1 = conv3x3_transpose(gh2q, W2) * (a1 > 0) * m
    dW1 = conv3x3_weight_grad(z[None], gh1)
    return loss, [dW1, dW2, dW3]


def adam_step(Ws, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) of FP64 master weights; state = (m, v, t)."""
    m, v, t = state
    t += 1
    out = []
    for k, (W, g) in enumerate(zip(Ws, grads)):
        m[k] = b1 * m[k] + (1 - b1) * g
        v[k] = b2 * v[k] + (1 - b2) * g * g
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        out.append(W - lr * mh / (np.sqrt(vh) + eps))
    return out, (m, v, t)
