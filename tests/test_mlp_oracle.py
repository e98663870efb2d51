"""Pins for the FP64 network oracle (oracle/mlp.py): finite differences, an
independent autograd implementation (torch CPU float64), Adam's closed forms
(first step; a constant gradient over many steps, where bias correction makes
every step -lr g/(|g|+eps)), the input normalisation's fixed points and
period, the BF16 rounding points, and SiLU identities."""
import numpy as np
import pytest
import torch

import fieldgen as fg
from tests.oracle_under_test import mlp

RNG = np.random.default_rng(7)


def rand_params(widths):
    return [(RNG.normal(size=(widths[i + 1], widths[i])) / np.sqrt(widths[i]),
             RNG.normal(size=widths[i + 1]) * 0.1) for i in range(len(widths) - 1)]


def test_silu_and_derivative():
    z = np.linspace(-8, 8, 1001)
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(mlp.silu(np.array([30.0])), [30.0], rtol=1e-12)
    e = 1e-6
    np.testing.assert_allclose(mlp.dsilu(z), (mlp.silu(z + e) - mlp.silu(z - e)) / (2 * e), atol=1e-8)


def test_gradients_match_central_differences():
    widths = (3, 5, 4, 3)
    params = rand_params(widths)
    x = RNG.uniform(-1, 1, size=(7, 3))
    sigma = np.array([0.5, 1.5, 2.0])
    tgt = RNG.normal(size=(7, 3))
    out, cache = mlp.forward(params, x, sigma)
    grads = mlp.backward(params, cache, out, tgt, sigma)
    e = 1e-6
    for l in range(len(params)):
        for k in range(2):
            p = params[l][k]
            num = np.zeros_like(p)
            for idx in np.ndindex(p.shape):
                old = p[idx]
                p[idx] = old + e
                lp = mlp.loss(mlp.forward(params, x, sigma)[0], tgt, sigma)
                p[idx] = old - e
                lm = mlp.loss(mlp.forward(params, x, sigma)[0], tgt, sigma)
                p[idx] = old
                num[idx] = (lp - lm) / (2 * e)
            np.testing.assert_allclose(grads[l][k], num, rtol=1e-6, atol=1e-9)


def test_full_width_network_matches_torch_autograd():
    params = [(w.astype(np.float64), b.astype(np.float64)) for w, b in fg.mlp_init()]
    assert mlp.n_params() == 199171 == sum(w.size + b.size for w, b in params)
    x = RNG.uniform(-1, 1, size=(64, 3))
    sigma = np.array([0.2, 0.3, 0.25])
    tgt = RNG.normal(size=(64, 3)) * 0.2
    out, cache = mlp.forward(params, x, sigma)
    grads = mlp.backward(params, cache, out, tgt, sigma)
    tp = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True)) for w, b in params]
    h = torch.tensor(x)
    for l, (W, b) in enumerate(tp):
        z = h @ W.T + b
        h = torch.nn.functional.silu(z) if l < len(tp) - 1 else z
    o = h * torch.tensor(sigma)
    L = (((o - torch.tensor(tgt)) / torch.tensor(sigma)) ** 2).mean()
    L.backward()
    np.testing.assert_allclose(out, o.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert abs(mlp.loss(out, tgt, sigma) - L.item()) < 1e-12
    for (W, b), (gw, gb) in zip(tp, grads):
        np.testing.assert_allclose(gw, W.grad.numpy(), rtol=1e-9, atol=1e-14)
        np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_adam_first_step_closed_form():
    params = rand_params((3, 4, 3))
    grads = [(RNG.normal(size=W.shape), RNG.normal(size=b.shape)) for W, b in params]
    m, v = mlp.zeros_like(params), mlp.zeros_like(params)
    before = [(W.copy(), b.copy()) for W, b in params]
    lr, eps = 1e-3, 1e-8
    mlp.adam_step(params, grads, m, v, 1, lr, eps=eps)
    for (W0, b0), (W1, b1), (gw, gb) in zip(before, params, grads):
        # after one step m_hat = g and v_hat = g^2: the update is -lr g / (|g| + eps)
        np.testing.assert_allclose(W1 - W0, -lr * gw / (np.abs(gw) + eps), rtol=1e-12, atol=1e-16)
        np.testing.assert_allclose(b1 - b0, -lr * gb / (np.abs(gb) + eps), rtol=1e-12, atol=1e-16)


def test_bf16_rounding_is_round_to_nearest_even():
    x = RNG.normal(size=10000).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.round_bf16(x), ref)


def test_adam_constant_gradient_closed_form_over_many_steps():
    """With a constant gradient g, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    bias-corrected moments are g and g^2 at every t and each step moves by
    -lr g / (|g| + eps): after t steps p_t = p_0 - t lr g / (|g| + eps)."""
    params = rand_params((3, 4, 3))
    grads = [(RNG.normal(size=W.shape) * 10.0 ** RNG.integers(-3, 2, size=W.shape),
              RNG.normal(size=b.shape)) for W, b in params]
    m, v = mlp.zeros_like(params), mlp.zeros_like(params)
    before = [(W.copy(), b.copy()) for W, b in params]
    lr, eps = 1e-3, 1e-8
    for t in range(1, 8):
        mlp.adam_step(params, grads, m, v, t, lr, eps=eps)
        for (W0, b0), (W1, b1), (gw, gb) in zip(before, params, grads):
            np.testing.assert_allclose(W1 - W0, -t * lr * gw / (np.abs(gw) + eps), rtol=1e-9, atol=1e-15)
            np.testing.assert_allclose(b1 - b0, -t * lr * gb / (np.abs(gb) + eps), rtol=1e-9, atol=1e-15)


def test_adam_second_step_after_a_sign_flip():
    """g then -g: m_2 = 0.09 g - 0.1 g = -0.01 g, v_2 = 0.001999 g^2 (b2 = 0.999), so the
    second step moves by -lr (-0.01 g / 0.19) / (sqrt(0.001999 g^2 / 0.001999) + eps)."""
    p = [(np.array([[0.5, -2.0]]), np.array([0.25]))]
    g = np.array([[0.3, -4.0]]), np.array([2.0])
    m, v = mlp.zeros_like(p), mlp.zeros_like(p)
    lr, eps = 1e-2, 1e-8
    mlp.adam_step(p, [g], m, v, 1, lr, eps=eps)
    p1 = p[0][0].copy()
    mlp.adam_step(p, [(-g[0], -g[1])], m, v, 2, lr, eps=eps)
    mhat = (0.9 * 0.1 * g[0] - 0.1 * g[0]) / (1 - 0.9 ** 2)
    vhat = (0.999 * 0.001 * g[0] ** 2 + 0.001 * g[0] ** 2) / (1 - 0.999 ** 2)
    np.testing.assert_allclose(p[0][0] - p1, -lr * mhat / (np.sqrt(vhat) + eps), rtol=1e-12)


def test_normalise_maps_each_period_onto_minus_one_to_one():
    L = 2 * np.pi
    x = np.array([0.0, L / 2, L / 4, 3 * L / 4, L - 1e-12])
    np.testing.assert_allclose(mlp.normalise(x, L), [-1.0, 0.0, -0.5, 0.5, 1.0], atol=1e-11)
    y = RNG.uniform(-3 * L, 3 * L, size=1000)
    np.testing.assert_allclose(mlp.normalise(y + 2 * L, L), mlp.normalise(y, L), atol=1e-12)
    assert (mlp.normalise(y, L) >= -1).all() and (mlp.normalise(y, L) < 1).all()


def test_forward_rounds_hidden_activations_where_asked():
    params = rand_params((3, 16, 16, 3))
    x = RNG.uniform(-1, 1, size=(50, 3))
    sigma = np.ones(3)
    plain, (hs, _) = mlp.forward(params, x, sigma)
    rounded, (hr, _) = mlp.forward(params, x, sigma, round_act=mlp.round_bf16)
    for h in hr[1:]:  # every hidden activation is a BF16 value
        np.testing.assert_array_equal(h, torch.from_numpy(h).to(torch.bfloat16).to(torch.float64).numpy())
    np.testing.assert_array_equal(hr[0], x)  # the input is the caller's
    assert 0 < np.abs(rounded - plain).max() < 0.05 * np.abs(plain).max()
