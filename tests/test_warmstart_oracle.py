"""Pins of the warm-start reference (POD, perceptron, Adam) against facts
that do not come from the reference itself: LAPACK's SVD, the
Eckart-Young theorem, a network small enough to evaluate by hand, central
finite differences and the closed form of Adam under a constant gradient."""
import math

import numpy as np
import pytest

from oracle import warmstart as ws


def _snapshots(N=300, M=40, seed=0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((N, M)))
    V, _ = np.linalg.qr(rng.standard_normal((M, M)))
    s = 10.0 ** -np.linspace(0, 6, M)          # decaying spectrum
    return (U * s) @ V.T, s


def test_pod_equals_svd_and_eckart_young():
    S, s = _snapshots()
    m = 12
    Phi, sigma = ws.pod_basis(S, m)
    np.testing.assert_allclose(sigma, s[:m], rtol=1e-8)
    np.testing.assert_allclose(Phi.T @ Phi, np.eye(m), atol=1e-8)
    U = np.linalg.svd(S, full_matrices=False)[0][:, :m]
    np.testing.assert_allclose(np.abs(np.sum(U * Phi, axis=0)), 1.0, atol=1e-8)   # same modes up to sign
    # best rank-m approximation error (Eckart-Young)
    R = S - Phi @ ws.pod_project(Phi, S)
    assert abs(np.linalg.norm(R) - np.sqrt(np.sum(s[m:] ** 2))) <= 1e-8 * np.linalg.norm(S)
    # expand(project(x)) is the identity on the span
    c = np.random.default_rng(1).standard_normal((m, 3))
    np.testing.assert_allclose(ws.pod_project(Phi, ws.pod_expand(Phi, c)), c, atol=1e-10)


def test_mlp_forward_by_hand():
    sizes = [1, 1, 1]
    w1, b1, w2, b2 = 0.7, -0.2, 1.5, 0.3
    p = np.array([w1, b1, w2, b2])
    X = np.array([[-1.0], [0.0], [2.5]])
    Y = ws.mlp_forward(p, sizes, X)
    for x, y in zip(X[:, 0], Y[:, 0]):
        assert y == pytest.approx(w2 * math.tanh(w1 * x + b1) + b2, abs=1e-15)
    # two inputs, two hidden units, one output: weights row-major (out x in)
    sizes = [2, 2, 1]
    p = np.array([1.0, 2.0, 3.0, 4.0, 0.1, 0.2, 0.5, -1.0, 0.05])
    x = np.array([[0.3, -0.4]])
    h = [math.tanh(1.0 * 0.3 + 2.0 * -0.4 + 0.1), math.tanh(3.0 * 0.3 + 4.0 * -0.4 + 0.2)]
    assert ws.mlp_forward(p, sizes, x)[0, 0] == pytest.approx(0.5 * h[0] - 1.0 * h[1] + 0.05, abs=1e-15)


def test_mlp_gradient_matches_finite_differences():
    sizes = [3, 7, 5, 4]
    rng = np.random.default_rng(2)
    n = ws.param_count(sizes)
    assert n == 7 * 3 + 7 + 5 * 7 + 5 + 4 * 5 + 4
    p = rng.standard_normal(n) * 0.5
    X = rng.standard_normal((6, 3))
    T = rng.standard_normal((6, 4))
    w = rng.uniform(0.5, 2.0, 4)
    loss, g = ws.mlp_loss_grad(p, sizes, X, T, w)
    Y = ws.mlp_forward(p, sizes, X)
    assert loss == pytest.approx(0.5 * np.sum(w * (Y - T) ** 2) / 6, rel=1e-14)
    h = 1e-6
    fd = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd[i] = (ws.mlp_loss_grad(p + e, sizes, X, T, w)[0] - ws.mlp_loss_grad(p - e, sizes, X, T, w)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves theta by lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 7.0])
    th0 = np.array([1.0, 2.0, 3.0, 4.0])
    opt = ws.Adam(4, lr=0.01, eps=1e-8)
    th = th0.copy()
    for t in range(1, 6):
        th = opt.step(th, g)
        np.testing.assert_allclose(th, th0 - t * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_minimises_a_quadratic():
    A = np.diag([1.0, 10.0, 100.0])
    x = np.array([1.0, -1.0, 0.5])
    opt = ws.Adam(3, lr=0.05)
    for _ in range(2000):
        x = opt.step(x, A @ x)
    assert np.linalg.norm(x) < 1e-3


def test_sun_features():
    e = np.deg2rad([5.0, 30.0, 17.5])
    az = np.deg2rad([90.0, 180.0, 0.0])
    suns = np.column_stack([np.cos(e) * np.cos(az), np.cos(e) * np.sin(az), np.sin(e)])
    f = ws.sun_features(suns)
    np.testing.assert_allclose(f, [[0, 1, -1], [-1, 0, 1], [1, 0, 0]], atol=1e-12)
