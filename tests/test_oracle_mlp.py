"""Pins of the FP64 network reference: finite differences for the gradient,
closed forms for the loss, SiLU and the first Adam steps, and BF16 rounding
of known values."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from paper_1810_01780_amd import workloads as W


def _batch(B, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, 5))
    t = rng.standard_normal((B, 8))
    m = (rng.random((B, 4)) < 0.6).astype(np.float64)
    return x, t, m


def test_param_count_and_generator():
    assert M.param_count() == 5 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 12 + 12 == 201996
    p = W.mlp_init_params(3)
    assert p.dtype == np.float32 and p.shape == (201996,)
    assert np.array_equal(p, W.mlp_init_params(3)) and not np.array_equal(p, W.mlp_init_params(4))


def test_round_bf16_known_values():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.0e-30, 65504.0],
                 dtype=np.float32)
    r = M.round_bf16(v)
    # 8 significant bits; ties go to the even neighbour
    assert r.tolist() == [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, r[5], 65536.0]
    assert abs(r[5] - 3.0e-30) <= 3.0e-30 * 2 ** -8


def test_silu_and_its_derivative():
    z = np.linspace(-8, 8, 101)
    assert np.allclose(M.silu(z), z * 0.5 * (1 + np.tanh(z / 2)), rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.allclose(M.silu_grad(z), fd, rtol=1e-8, atol=1e-10)


def test_loss_closed_forms():
    B = 7
    y = np.zeros((B, 12))
    t = np.zeros((B, 8))
    m = np.ones((B, 4))
    # zero logits: four cross-entropies of log 2 per row, no regression error
    assert M.loss(y, t, m) == pytest.approx(4 * math.log(2), rel=1e-15)
    t[:, 1] = 3.0
    m[:, 1] = 0.0
    # masked family 1 does not count; family 0 adds 3^2
    assert M.loss(y, t, m) == pytest.approx(4 * math.log(2) + 9.0, rel=1e-15)
    # a several-roots logit z with label 1 costs log(1 + e^-z), with label 0
    # log(1 + e^z)
    y[:, 11] = 2.0
    m[:, 3] = 1.0
    l1 = M.loss(y, t, m)
    m[:, 3] = 0.0
    l0 = M.loss(y, t, m)
    assert l1 == pytest.approx(3 * math.log(2) + 9.0 + math.log1p(math.exp(-2.0)), rel=1e-15)
    assert l0 == pytest.approx(3 * math.log(2) + 9.0 + math.log1p(math.exp(2.0)), rel=1e-15)


def test_gradient_matches_finite_differences():
    """Central differences of the FP64 loss (without BF16 rounding) against
    the backpropagated gradient, on all output-layer parameters and a random
    sample of the others."""
    x, t, m = _batch(6, seed=1)
    p = W.mlp_init_params(1).astype(np.float64)
    p[-12:] = np.random.default_rng(2).standard_normal(12)  # non-zero output biases
    _, g = M.gradients(p, x, t, m, bf16=False)
    lay, total = M.layout()
    rng = np.random.default_rng(3)
    idx = np.concatenate([np.arange(lay[4][0], total),  # output layer
                          rng.choice(lay[4][0], 300, replace=False)])
    h = 1e-6
    for i in idx:
        pp = p.copy()
        pp[i] += h
        lp = M.loss(M.forward(pp, x, bf16=False)[0], t, m)
        pp[i] -= 2 * h
        lm = M.loss(M.forward(pp, x, bf16=False)[0], t, m)
        fd = (lp - lm) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-8), i


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(0)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    p1, m1, v1 = M.adam(p, np.zeros(50), np.zeros(50), g, 1, lr, eps=eps)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # a constant gradient keeps the step at lr sign(g) (up to eps)
    p2, _, _ = M.adam(p1, m1, v1, g, 2, lr, eps=eps)
    assert np.allclose(p2 - p1, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_bf16_evaluation_point():
    """With BF16 rounding the network is the FP64 network at rounded weights
    and inputs."""
    x, t, m = _batch(5, seed=4)
    p = W.mlp_init_params(2)
    pr = p.astype(np.float64)
    lay, _ = M.layout()
    for w, b, ni, no in lay:
        pr[w:w + ni * no] = M.round_bf16(p[w:w + ni * no])
    y1, _ = M.forward(p, x, bf16=True)
    y2, _ = M.forward(pr, M.round_bf16(x), bf16=False)
    assert np.array_equal(y1, y2)
