"""Pins of the FP64 learned-guess reference (CPU)."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import mlp_ref as M
import workloads as W


def test_param_count():
    assert M.NPARAM == 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1 == 4801


def test_gradient_vs_central_differences():
    rng = np.random.default_rng(0)
    theta = M.init(1) + 0.05 * rng.standard_normal(M.NPARAM)
    X = rng.standard_normal((37, 8))
    t = rng.standard_normal(37)
    g = M.grad(theta, X, t)
    idx = rng.choice(M.NPARAM, 300, replace=False)
    idx = np.concatenate([idx, [M.NPARAM - 1, 0, 512, 512 + 64]])   # b3, W1, b1, W2 corners
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss(theta + e, X, t) - M.loss(theta - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])), (i, fd, g[i])


def test_forward_is_the_plain_definition_on_one_sample():
    rng = np.random.default_rng(2)
    theta = M.init(3)
    x = rng.standard_normal(8)
    p = M.unpack(theta)
    h1 = [np.tanh(sum(p["W1"][i, k] * x[k] for k in range(8)) + p["b1"][i]) for i in range(64)]
    h2 = [np.tanh(sum(p["W2"][i, k] * h1[k] for k in range(64)) + p["b2"][i]) for i in range(64)]
    y = sum(p["w3"][i] * h2[i] for i in range(64)) + p["b3"][0]
    assert abs(M.forward(theta, x)[0] - y) < 1e-12


def test_target_and_guess_invert_and_stay_admissible():
    inp, eos = W.riemann_problem_set(5, 2000)
    plo, P = M.scales(inp, eos)
    for i in range(0, 2000, 97):
        rc, out, _ = oracle.riemann(inp[i], eos[i])
        if rc != oracle.OK:
            continue
        y = M.target(out[0], inp[i:i + 1], eos[i:i + 1])
        assert abs(M.guess(y, inp[i:i + 1], eos[i:i + 1])[0] - out[0]) <= 1e-12 * (out[0] - plo[i])
    # any output, however wild, maps to an admissible pressure
    g = M.guess(np.array([-700.0] * 3 + [40.0] * 3), inp[:6], eos[:6])
    assert np.all(g >= plo[:6])


def test_features_symmetries():
    """Swapping the two sides (with u -> -u) negates the antisymmetric
    features; equal states give zero features."""
    inp, eos = W.riemann_problem_set(6, 50)
    X = M.features(inp, eos)
    sw = np.stack([inp[:, 3], -inp[:, 4], inp[:, 5], inp[:, 0], -inp[:, 1], inp[:, 2]], axis=1)
    se = np.stack([eos[:, 2], eos[:, 3], eos[:, 0], eos[:, 1]], axis=1)
    Xs = M.features(sw, se)
    assert np.allclose(Xs[:, [0, 1]], X[:, [1, 0]], atol=1e-14)
    assert np.allclose(Xs[:, [4, 5]], X[:, [5, 4]], atol=1e-12)
    assert np.allclose(Xs[:, 6], -X[:, 6], atol=1e-14)
    assert np.allclose(Xs[:, 7], -X[:, 7], atol=1e-14)
    same = np.array([[1000.0, 3.0, 2e5, 1000.0, 3.0, 2e5]])
    e = np.array([[6.12, 3.43e8, 6.12, 3.43e8]])
    assert np.allclose(M.features(same, e), 0.0, atol=1e-15)


def test_adam_reduces_loss_on_a_small_problem():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((256, 8))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 4]
    theta = M.init(0)
    m = np.zeros(M.NPARAM)
    v = np.zeros(M.NPARAM)
    l0 = M.loss(theta, X, t)
    for s in range(1, 301):
        theta, m, v = M.adam_step(theta, M.grad(theta, X, t), m, v, s, lr=3e-3)
    assert M.loss(theta, X, t) < 0.1 * l0
