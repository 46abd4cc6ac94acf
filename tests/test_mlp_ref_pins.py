"""Pins of the float64 scheduler-network reference (``oracle.mlp_ref``).

* gradients against central finite differences of the loss (a different
  computation from back-propagation);
* closed forms: zero weights give the output bias; with all pre-activations
  positive the network is the affine map W3 W2 W1 x + (W3 W2 b1 + W3 b2 + b3);
  an empty mask gives zero loss and gradient; the first Adam step moves each
  parameter by lr * g / (|g| + eps) (bias-corrected moments equal g and g^2);
* an invariant: Adam on a fixed batch drives the loss down.
"""
import numpy as np
import pytest

from oracle import mlp_ref as M

F, H, P = 9, 32, 3


def rand_theta(rng, scale=0.3):
    return rng.normal(0, scale, size=M.n_params(F, H, P))


def test_gradient_matches_finite_differences(rng):
    X = rng.normal(0, 1, size=(40, F))
    T = rng.normal(0, 1, size=(40, P))
    Mk = (rng.random((40, P)) < 0.7).astype(np.float64)
    th = rand_theta(rng)
    L, g = M.loss_and_grad(th, X, T, Mk, F, H, P)
    assert abs(L - M.loss(th, X, T, Mk, F, H, P)) < 1e-12
    eps = 1e-6
    idx = rng.choice(len(th), size=200, replace=False)
    for i in idx:
        tp = th.copy(); tp[i] += eps
        tm = th.copy(); tm[i] -= eps
        fd = (M.loss(tp, X, T, Mk, F, H, P) - M.loss(tm, X, T, Mk, F, H, P)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_zero_weights_give_output_bias(rng):
    th = np.zeros(M.n_params(F, H, P))
    W1, b1, W2, b2, W3, b3 = M.unpack(th, F, H, P)
    th[-P:] = [1.5, -2.0, 0.25]
    y = M.forward(th, rng.normal(size=(5, F)), F, H, P)
    np.testing.assert_array_equal(y, np.tile([1.5, -2.0, 0.25], (5, 1)))


def test_positive_regime_is_affine(rng):
    W1 = rng.random((H, F)); b1 = rng.random(H)
    W2 = rng.random((H, H)); b2 = rng.random(H)
    W3 = rng.normal(size=(P, H)); b3 = rng.normal(size=P)
    th = M.pack(W1, b1, W2, b2, W3, b3)
    X = rng.random((7, F))
    A = W3 @ W2 @ W1
    c = W3 @ W2 @ b1 + W3 @ b2 + b3
    np.testing.assert_allclose(M.forward(th, X, F, H, P), X @ A.T + c, rtol=1e-12)


def test_empty_mask(rng):
    th = rand_theta(rng)
    L, g = M.loss_and_grad(th, rng.normal(size=(4, F)), np.zeros((4, P)), np.zeros((4, P)), F, H, P)
    assert L == 0.0 and not g.any()


def test_first_adam_step_closed_form(rng):
    th = rand_theta(rng)
    g = rng.normal(size=th.shape)
    lr, eps = 1e-3, 1e-8
    th1, m1, v1 = M.adam_step(th, g, np.zeros_like(th), np.zeros_like(th), 1, lr, eps=eps)
    np.testing.assert_allclose(th1, th - lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.001 * g * g)


def test_adam_steps_two_and_three_by_hand():
    """Adam at t = 2 and t = 3 against values worked out by hand (Kingma and
    Ba, Algorithm 1) for beta1 = 1/2, beta2 = 3/4, lr = 1, eps = 0 and the
    gradients 2, 1, -2 (one scalar parameter, replicated with three starting
    values).  The bias corrections divide by 1 - beta**t, so t = 2 and t = 3
    tell apart a correction by beta instead of beta**t (which would give a
    step of exactly 1 at t = 2)."""
    th0 = np.array([0.0, 1.5, -3.0])
    z = np.zeros(3)
    kw = dict(beta1=0.5, beta2=0.75, eps=0.0)
    # t = 1: m1 = 1, v1 = 1, mhat = 2, vhat = 4, step 1
    th1, m1, v1 = M.adam_step(th0, np.full(3, 2.0), z, z, 1, 1.0, **kw)
    np.testing.assert_allclose(m1, 1.0)
    np.testing.assert_allclose(v1, 1.0)
    np.testing.assert_allclose(th1, th0 - 1.0)
    # t = 2, g = 1: m2 = 1, v2 = 1, mhat = 1/(3/4) = 4/3,
    # vhat = 1/(7/16) = 16/7, step = (4/3) / (4/sqrt 7) = sqrt(7)/3
    th2, m2, v2 = M.adam_step(th1, np.full(3, 1.0), m1, v1, 2, 1.0, **kw)
    np.testing.assert_allclose(m2, 1.0)
    np.testing.assert_allclose(v2, 1.0)
    np.testing.assert_allclose(th2, th1 - np.sqrt(7.0) / 3.0, rtol=1e-14)
    # t = 3, g = -2: m3 = 1/2 - 1 = -1/2, v3 = 3/4 + 1 = 7/4,
    # mhat = (-1/2)/(7/8) = -4/7, vhat = (7/4)/(37/64) = 112/37,
    # step = (-4/7) / sqrt(112/37)
    th3, m3, v3 = M.adam_step(th2, np.full(3, -2.0), m2, v2, 3, 1.0, **kw)
    np.testing.assert_allclose(m3, -0.5)
    np.testing.assert_allclose(v3, 1.75)
    np.testing.assert_allclose(th3, th2 + (4.0 / 7.0) / np.sqrt(112.0 / 37.0), rtol=1e-14)


def test_adam_reduces_loss(rng):
    X = rng.normal(size=(256, F))
    true_w = rng.normal(size=(P, F))
    T = X @ true_w.T
    Mk = np.ones((256, P))
    th = rand_theta(rng, 0.2)
    m = np.zeros_like(th); v = np.zeros_like(th)
    L0 = M.loss(th, X, T, Mk, F, H, P)
    for t in range(1, 401):
        _, g = M.loss_and_grad(th, X, T, Mk, F, H, P)
        th, m, v = M.adam_step(th, g, m, v, t, 3e-3)
    assert M.loss(th, X, T, Mk, F, H, P) < 0.1 * L0


def test_f32_forward_close_to_f64(rng):
    th = rand_theta(rng)
    X = rng.normal(size=(64, F))
    np.testing.assert_allclose(M.forward_f32(th, X, F, H, P), M.forward(th, X, F, H, P),
                               rtol=1e-4, atol=1e-4)


def test_bad_length_rejected():
    with pytest.raises(ValueError):
        M.unpack(np.zeros(10), F, H, P)


def test_relu_gate_option():
    """Fixed gates equal to the network's own decisions change nothing; all
    gates closed leave only the output bias (y = b3), so every gradient but
    db3 vanishes."""
    rng = np.random.default_rng(11)
    F, H, P = 9, 32, 3
    th = rng.normal(0, 0.4, M.n_params(F, H, P))
    X = rng.normal(size=(40, F))
    T = rng.normal(size=(40, P))
    Mk = (rng.random((40, P)) < 0.7).astype(float)
    _, (_, a1, _, a2, _) = M.forward(th, X, F, H, P, keep=True)
    L0, g0 = M.loss_and_grad(th, X, T, Mk, F, H, P)
    L1, g1 = M.loss_and_grad(th, X, T, Mk, F, H, P, relu_gate=(a1 > 0, a2 > 0))
    assert L0 == L1 and np.array_equal(g0, g1)
    closed = (np.zeros_like(a1, dtype=bool), np.zeros_like(a2, dtype=bool))
    L2, g2 = M.loss_and_grad(th, X, T, Mk, F, H, P, relu_gate=closed)
    b3 = M.unpack(th, F, H, P)[5]
    d = np.where(Mk > 0, b3 - T, 0.0)
    assert L2 == pytest.approx(float((Mk * d * d).sum() / Mk.sum()))
    assert np.all(g2[:-P] == 0.0)
    assert np.allclose(g2[-P:], (2.0 * Mk * d / Mk.sum()).sum(axis=0))
