"""Pins of the oracle's learned-smoother network (forward, adjoints, gradients)."""
import numpy as np
import pytest

from oracle import learned as ln


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6))
    W = rng.standard_normal((3, 2, 3, 3))
    y = ln.conv3x3(x, W)
    for o in range(3):
        for j in range(5):
            for i in range(6):
                s = 0.0
                for c in range(2):
                    for dy in range(3):
                        for dx in range(3):
                            jj, ii = j + dy - 1, i + dx - 1
                            if 0 <= jj < 5 and 0 <= ii < 6:
                                s += W[o, c, dy, dx] * x[c, jj, ii]
                assert abs(y[o, j, i] - s) < 1e-12


def test_transpose_is_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 7, 6))
    g = rng.standard_normal((3, 7, 6))
    W = rng.standard_normal((3, 4, 3, 3))
    lhs = np.sum(ln.conv3x3(x, W) * g)
    assert abs(lhs - np.sum(x * ln.conv3x3_transpose(g, W))) < 1e-10
    dW = ln.conv3x3_weight_grad(x, g)
    assert abs(lhs - np.sum(dW * W)) < 1e-10


def test_positive_homogeneity():
    rng = np.random.default_rng(2)
    Ws = ln.init_weights(rng)
    z = rng.standard_normal((9, 9))
    y1, _ = ln.forward(z, Ws, bf16_points=False)
    y2, _ = ln.forward(3.5 * z, Ws, bf16_points=False)
    np.testing.assert_allclose(y2, 3.5 * y1, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("masked", [False, True])
def test_gradients_by_central_differences(masked):
    rng = np.random.default_rng(3)
    Ws = ln.init_weights(rng, channels=4)
    z = rng.standard_normal((8, 7))
    t = rng.standard_normal((8, 7))
    mask = np.ones((8, 7))
    lmask = np.ones((8, 7))
    if masked:
        mask[:, -2:] = 0.0
        lmask[:2, :] = 0.0
    loss, grads = ln.loss_and_grads(z, t, Ws, mask, lmask, bf16_points=False)
    h = 1e-6
    for k in range(3):
        for idx in [tuple(rng.integers(0, s) for s in Ws[k].shape) for _ in range(6)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[k][idx] += h
            Wm[k][idx] -= h
            lp, _ = ln.loss_and_grads(z, t, Wp, mask, lmask, bf16_points=False)
            lm_, _ = ln.loss_and_grads(z, t, Wm, mask, lmask, bf16_points=False)
            fd = (lp - lm_) / (2 * h)
            assert abs(fd - grads[k][idx]) <= 1e-6 * max(1.0, abs(fd))


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 1e-3])
    r = ln.bf16_round(vals)
    assert r[0] == 1.0 and r[3] == -2.5 and r[4] == 0.0
    assert r[1] == 1.0          # halfway: ties to even
    assert r[2] == 1.0 + 2 ** -7
    assert abs(r[5] - 1e-3) / 1e-3 < 2 ** -8


def test_adam_reduces_loss():
    rng = np.random.default_rng(4)
    Ws = ln.init_weights(rng, channels=4)
    z = rng.standard_normal((10, 10))
    t = 0.5 * z
    st = ([np.zeros_like(w) for w in Ws], [np.zeros_like(w) for w in Ws], 0)
    l0, _ = ln.loss_and_grads(z, t, Ws, bf16_points=False)
    for _ in range(200):
        l, g = ln.loss_and_grads(z, t, Ws, bf16_points=False)
        Ws, st = ln.adam_step(Ws, g, st, lr=3e-3)
    assert l < 0.5 * l0


def test_adam_two_steps_closed_form():
    """Two Adam steps on one scalar weight, derived by hand from the update
    rule (first and second moment averages with bias correction):
    after gradients g1, g2 the corrected moments are
        m^ = (b1 g1 + g2) / (1 + b1),   v^ = (b2 g1^2 + g2^2) / (1 + b2),
    and after g1 alone they are g1 and g1^2, so the first step moves the
    weight by lr g1 / (|g1| + eps).  A missing bias correction, square root or
    (1 - beta) factor changes either step by a large factor."""
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    w0 = np.array([0.25])
    g1, g2 = np.array([3.0]), np.array([-0.5])
    st = ([np.zeros(1)], [np.zeros(1)], 0)
    (w1,), st = ln.adam_step([w0], [g1], st, lr=lr, b1=b1, b2=b2, eps=eps)
    step1 = lr * g1 / (abs(g1) + eps)
    np.testing.assert_allclose(w1, w0 - step1, rtol=0, atol=1e-15)
    (w2,), st = ln.adam_step([w1], [g2], st, lr=lr, b1=b1, b2=b2, eps=eps)
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 ** 2 + g2 ** 2) / (1 + b2)
    np.testing.assert_allclose(w2, w1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)
    assert st[2] == 2
    # constant gradient: every step moves the weight by lr sign(g) for |g| >> eps
    w = [np.array([1.0])]
    st = ([np.zeros(1)], [np.zeros(1)], 0)
    for k in range(5):
        w, st = ln.adam_step(w, [np.array([7.0])], st, lr=lr)
    np.testing.assert_allclose(w[0], 1.0 - 5 * lr, rtol=0, atol=1e-10)
