"""Pins for the FP64 jump oracle (oracle/surrogate.py), each fixed by a closed form:

* a zero network on a uniform flow: the big-step residual is the length of the
  16h step (16 h |c|_inf), the commutation residual is 0, and the jump does not
  move (the identity map commutes with every flow map);
* a network that returns the exact 16-step displacement of a uniform flow has
  zero residuals of both kinds and lands where 16 plain steps land;
* on a rotation (a field in the trilinear span, sampled exactly) the big-step
  residual of a zero network is |(M(16 h w) - I)(x - c)|_inf and the
  commutation residual of a constant network D is |(I - M(h w)) D|_inf, with
  M(t) = I + tJ + (tJ)^2/2 + (tJ)^3/6 + (tJ)^4/24 the RK4 propagator of J;
* a residual equal to the tolerance is accepted, a rejected jump is plain RK4
  (with its terminations), an accepted jump leaving the block is an exit, and an
  undefined reference step rejects;
* the network rounds its input and hidden activations to BF16 exactly where the
  matrix cores take them (checked with torch's own BF16 conversion).
"""
import math

import numpy as np
import pytest
import torch

import fieldgen as fg
import oracle
from tests.oracle_under_test import mlp as omlp
from tests.oracle_under_test import surrogate as osur

H = 0.125
C = (0.25, -0.5, 0.125)   # dyadic uniform flow: every RK4 operation is exact or nearly so
W = 0.0625                # rotation rate (dyadic: node values are exact in FP32)
XC = 8.0


def uniform_field():
    blk = fg.closed_form_block(lambda x, y, z: (0 * x + C[0], 0 * x + C[1], 0 * x + C[2]), (16, 16, 16))
    return oracle.Field.from_block(blk)


def rotation_field():
    blk = fg.closed_form_block(lambda x, y, z: (-W * (y - XC), W * (x - XC), 0 * z), (16, 16, 16))
    return oracle.Field.from_block(blk)


def const_net(D, sigma=(0.5, 0.25, 1.0)):
    """All weights and hidden biases zero; the output bias makes sigma * b = D exactly."""
    sig = np.asarray(sigma, np.float64)
    widths = (3, 256, 256, 256, 256, 3)
    params = [(np.zeros((widths[l + 1], widths[l])), np.zeros(widths[l + 1])) for l in range(5)]
    params[4] = (params[4][0], np.asarray(D, np.float64) / sig)
    return osur.Network(params, sig, 16.0)


def points(n=64, lo=5.0, hi=9.0, sub=0):
    rng = np.random.default_rng(100 + sub)
    return rng.uniform(lo, hi, size=(n, 3))


def rk4_propagator(t):
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    A = t * J
    return np.eye(2) + A + A @ A / 2 + A @ A @ A / 6 + A @ A @ A @ A / 24


def test_zero_network_big_step_residual_is_the_step_length():
    F, net, x = uniform_field(), const_net((0, 0, 0)), points()
    r, Y = osur.residual(F, net, x, H, kind=1)
    L = 16 * H * max(abs(c) for c in C)
    np.testing.assert_allclose(r, L, rtol=1e-14)
    np.testing.assert_array_equal(Y, x)
    acc = osur.jump(F, net, x, H, L * (1 + 1e-9), kind=1)
    assert acc["accept"].all()
    np.testing.assert_array_equal(acc["next_pos"], x)  # a zero jump does not move
    rej = osur.jump(F, net, x, H, L * (1 - 1e-9), kind=1)
    assert not rej["accept"].any()
    np.testing.assert_allclose(rej["next_pos"], x + 16 * H * np.array(C), rtol=0, atol=1e-13)
    assert (rej["steps"] == 16).all() and (rej["code"] == oracle.ACTIVE).all()


@pytest.mark.parametrize("field", [uniform_field, rotation_field])
def test_zero_network_passes_the_commutation_residual(field):
    """The identity map commutes with every flow map: a network that predicts no motion
    has commutation residual 0 and is accepted at any tolerance (a property of the
    residual's definition that the endpoint-error judge exposes)."""
    F, net, x = field(), const_net((0, 0, 0)), points(sub=1)
    r, Y = osur.residual(F, net, x, H, kind=0)
    np.testing.assert_array_equal(r, 0.0)
    out = osur.jump(F, net, x, H, 0.0, kind=0)  # r == tol is accepted
    assert out["accept"].all()
    np.testing.assert_array_equal(out["next_pos"], x)


def test_exact_network_has_zero_residuals_and_lands_on_plain_rk4():
    F, x = uniform_field(), points(sub=2)
    D = 16 * H * np.array(C)
    net = const_net(D)
    for kind in (0, 1):
        r, Y = osur.residual(F, net, x, H, kind=kind)
        assert np.abs(r).max() <= 1e-14
        out = osur.jump(F, net, x, H, 1e-12, kind=kind)
        assert out["accept"].all()
        plain = F.trace(x, H, 16, keep_verts=False)["final_pos"]
        np.testing.assert_allclose(out["next_pos"], plain, rtol=0, atol=1e-13)


def test_rotation_big_step_residual_closed_form():
    F, net, x = rotation_field(), const_net((0, 0, 0)), points(sub=3)
    r, _ = osur.residual(F, net, x, H, kind=1)
    M = rk4_propagator(16 * H * W)
    d = (M - np.eye(2)) @ (x[:, :2] - XC).T
    np.testing.assert_allclose(r, np.abs(d).max(axis=0), rtol=1e-12)


def test_constant_network_commutation_residual_closed_form():
    F, x = rotation_field(), points(sub=4)
    D = np.array([0.375, -0.25, 0.5])
    r, Y = osur.residual(F, const_net(D), x, H, kind=0)
    M = rk4_propagator(H * W)
    expect = np.abs((np.eye(2) - M) @ D[:2]).max()
    np.testing.assert_allclose(r, expect, rtol=1e-10)
    np.testing.assert_allclose(Y, x + D, rtol=0, atol=1e-15)


def test_rejected_jump_is_plain_rk4_and_may_terminate():
    F = uniform_field()
    x = np.array([[14.6, 7.0, 7.0], [3.0, 4.0, 5.0]])
    out = osur.jump(F, const_net((0, 0, 0)), x, H, 0.0, kind=1)  # r = 1 > 0: rejected
    plain = F.trace(x, H, 16, keep_verts=False)
    assert not out["accept"].any()
    np.testing.assert_array_equal(out["next_pos"], plain["final_pos"])
    # 14.6 + n/32 crosses the owned face x = 15 at step 13
    assert out["steps"][0] == 13 and out["code"][0] == oracle.EXIT
    assert out["steps"][1] == 16 and out["code"][1] == oracle.ACTIVE


def test_accepted_jump_leaving_the_block_exits():
    F = uniform_field()
    x = np.array([[14.6, 7.0, 7.0]])
    out = osur.jump(F, const_net(16 * H * np.array(C)), x, H, 1e-9, kind=0)
    assert out["accept"][0] and out["code"][0] == oracle.EXIT
    np.testing.assert_allclose(out["next_pos"][0], [15.1, 6.0, 7.25], rtol=0, atol=1e-12)


def test_undefined_reference_step_rejects():
    """The 16h step from x = 15.8 samples beyond the stored nodes (x <= 16): r = inf."""
    F = uniform_field()
    x = np.array([[15.8, 7.0, 7.0]])
    r, _ = osur.residual(F, const_net((0, 0, 0)), x, H, kind=1)
    assert np.isinf(r[0])
    assert not osur.jump(F, const_net((0, 0, 0)), x, H, 1e30, kind=1)["accept"][0]


def _bf16(v):
    return float(torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64))


def test_network_rounds_input_and_activations_to_bf16():
    """A chain network: unit weights carry x-hat through four SiLU layers along one
    hidden unit; the output is sigma * bf16(silu(...bf16(silu(bf16(xhat)))...))."""
    widths = (3, 256, 256, 256, 256, 3)
    params = [(np.zeros((widths[l + 1], widths[l])), np.zeros(widths[l + 1])) for l in range(5)]
    for l in range(5):
        params[l][0][0, 0] = 1.0
    sigma = (0.75, 1.0, 1.0)
    net = osur.Network(params, sigma, 2 * math.pi)
    xs = np.array([[0.3, 1.0, 2.0], [4.1, 0.0, 0.0], [7.9, 3.0, 3.0], [-0.7, 1.0, 1.0]])
    out = net(xs)
    for row, x in zip(out, xs[:, 0]):
        L = 2 * math.pi
        h = _bf16(2.0 * ((x % L) / L) - 1.0)
        for _ in range(4):
            h = _bf16(h / (1.0 + math.exp(-h)))
        assert row[0] == pytest.approx(sigma[0] * h, rel=1e-15, abs=0)
        assert row[1] == 0.0 and row[2] == 0.0


def test_bf16_weights_round_w_and_keep_b():
    params = fg.mlp_init(5)
    q = osur.bf16_weights(params)
    for (W0, b0), (W1, b1) in zip(params, q):
        np.testing.assert_array_equal(W1, torch.from_numpy(W0).to(torch.bfloat16).to(torch.float64).numpy())
        np.testing.assert_array_equal(b1, b0.astype(np.float64))
