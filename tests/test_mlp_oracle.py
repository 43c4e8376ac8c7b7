"""Pins of the float64 reference of the scheduler network (oracle/mlp_oracle.py)
against facts that do not come from its own code: central finite differences
of the forward pass, hand-evaluated small networks, the closed form of Adam's
first step, and the defining properties of the training targets."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M

F, H, O = 8, 16, 4


def _rand(seed, B=7):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.5, M.param_count(F, H, O))
    X = rng.normal(0, 1, (B, F))
    return rng, p, X


def test_backward_matches_finite_differences():
    rng, p, X = _rand(1)
    dY = rng.normal(0, 1, (X.shape[0], O))
    g = M.backward(p, X, dY, F, H, O)
    eps = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        num[i] = ((M.forward(p + e, X, F, H, O)[0] * dY).sum()
                  - (M.forward(p - e, X, F, H, O)[0] * dY).sum()) / (2 * eps)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-8)


def test_loss_gradient_matches_finite_differences():
    rng, p, X = _rand(2, B=11)
    T = rng.normal(0, 1, (11, O))
    Wt = rng.uniform(0, 2, (11, O))
    Wt[3, 1] = 0.0
    g = M.loss_grad(p, X, T, Wt, F, H, O)
    eps = 1e-6
    for i in range(0, p.size, 7):
        e = np.zeros_like(p)
        e[i] = eps
        num = (M.loss(p + e, X, T, Wt, F, H, O) - M.loss(p - e, X, T, Wt, F, H, O)) / (2 * eps)
        assert abs(g[i] - num) <= 1e-6 * max(1.0, abs(num))


def test_small_networks_by_hand():
    # F = 2, H = 1, O = 2: y_o = w2[o] * tanh(w1 . x + b1) + b2[o]
    p = np.array([0.5, -1.0, 0.25, 2.0, -3.0, 0.1, 0.2])
    x = np.array([[1.5, 0.5]])
    h = math.tanh(0.5 * 1.5 - 1.0 * 0.5 + 0.25)
    y, hid = M.forward(p, x, 2, 1, 2)
    assert abs(hid[0, 0] - h) < 1e-15
    assert abs(y[0, 0] - (2.0 * h + 0.1)) < 1e-15 and abs(y[0, 1] - (-3.0 * h + 0.2)) < 1e-15
    # zero output weights: the output is the bias, and no gradient reaches layer 1
    rng, p, X = _rand(3)
    W1, b1, W2, b2 = M.unpack(p, F, H, O)
    p0 = M.pack(W1, b1, np.zeros_like(W2), b2)
    np.testing.assert_array_equal(M.forward(p0, X, F, H, O)[0], np.tile(b2, (X.shape[0], 1)))
    g = M.backward(p0, X, np.ones((X.shape[0], O)), F, H, O)
    assert np.all(g[:H * F + H] == 0) and np.all(g[-O:] == X.shape[0])


def test_adam_first_step_is_signed_step():
    # from zero moments, the first bias-corrected step is lr * g / (|g| + eps)
    rng, p, X = _rand(4, B=9)
    T = rng.normal(0, 1, (9, O))
    Wt = np.ones((9, O))
    g = M.loss_grad(p, X, T, Wt, F, H, O)
    lr = 0.01
    p1, m1, v1 = M.adam_train(p, np.zeros_like(p), np.zeros_like(p), X, T, Wt, F, H, O, 1, 0, lr)
    np.testing.assert_allclose(p - p1, lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


def test_adam_fits_a_realisable_target():
    # a teacher network of the same shape generates the targets
    rng = np.random.default_rng(5)
    teacher = rng.normal(0, 0.7, M.param_count(F, H, O))
    X = rng.normal(0, 1, (200, F))
    T = M.forward(teacher, X, F, H, O)[0]
    Wt = np.ones_like(T)
    p0 = rng.normal(0, 0.3, teacher.size)
    l0 = M.loss(p0, X, T, Wt, F, H, O)
    p1, _, _ = M.adam_train(p0, np.zeros_like(p0), np.zeros_like(p0), X, T, Wt, F, H, O, 400, 0, 0.02)
    assert M.loss(p1, X, T, Wt, F, H, O) < l0 / 20


def test_sched_prep_definition():
    X = np.array([[1.0, 5.0], [3.0, 5.0], [5.0, 5.0]])
    T = np.array([[1.0, 2.0, 0.0], [4.0, 8.0, 16.0], [-1.0, 0.0, 0.0]])
    mu, isd, xn, Y, Wt = M.sched_prep(X, T)
    np.testing.assert_allclose(mu, [3.0, 5.0])
    # std of (1, 3, 5) is sqrt(8/3); a constant feature gets 1 / 1e-3
    np.testing.assert_allclose(isd, [1 / math.sqrt(8 / 3), 1e3])
    np.testing.assert_allclose(xn[:, 1], 0.0)
    np.testing.assert_allclose(Y[0], [0.0, 1.0, 0.0])
    np.testing.assert_allclose(Y[1], [2.0, 3.0, 4.0])
    # row maxima 2 and 16 (the third row has no measurement), mean 9
    np.testing.assert_allclose(Wt[0], [2 / 9, 2 / 9, 0.0])
    np.testing.assert_allclose(Wt[1], [16 / 9] * 3)
    assert np.all(Wt[2] == 0)


def test_model_scores_apply_normalisation():
    rng, p, X = _rand(6)
    mu = rng.normal(0, 1, F)
    isd = rng.uniform(0.5, 2, F)
    part = np.concatenate([[1205.0, F, H, O], mu, isd, p])
    np.testing.assert_allclose(M.model_scores(part, X), M.forward(p, (X - mu) * isd, F, H, O)[0], rtol=1e-14)
