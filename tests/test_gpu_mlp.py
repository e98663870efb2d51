"""GPU network kernels (BF16 MFMA, FP32 accumulate) against the FP64 network
oracle on the same BF16-rounded weights and inputs."""
import sys

import numpy as np
import pytest

import fieldgen as fg
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_02627_amd as S
    S._load()
    return S


def bf16_params(params):
    return [(omlp.round_bf16(W), b.astype(np.float64)) for W, b in params]


def rel_frob(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_forward_matches_oracle(S):
    import torch
    note("mlp forward")
    params = fg.mlp_init(5)
    sigma = np.array([0.2, 0.3, 0.25])
    m = S.streami_mlp_create(params, sigma, 2 * np.pi)
    rng = np.random.default_rng(3)
    for n in (1, 33, 1000, 70000):  # ragged vs the 32-row tiles, several chunks of waves
        x = rng.uniform(-7, 13, size=(n, 3)).astype(np.float32)
        xd = torch.from_numpy(x).cuda()
        out = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
        S.streami_mlp_forward(m, xd, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        xhat = omlp.round_bf16(omlp.normalise(x, 2 * np.pi))
        ref, _ = omlp.forward(bf16_params(params), xhat, sigma)
        assert rel_frob(got, ref) < 1e-2, (n, rel_frob(got, ref))
        cos = np.sum(got * ref) / np.linalg.norm(got) / np.linalg.norm(ref)
        assert cos > 0.9999, cos
    S.streami_mlp_destroy(m)


def test_gradients_match_oracle(S):
    """Gradients against the oracle that rounds only the weights and the input to BF16, not the
    hidden activations or back-propagated gradients.  The kernels round each of the four hidden
    layers' activations and each layer's incoming gradient to BF16 (relative error up to 2^-9
    each, about 2^-9/sqrt(3) rms); summed over the eight rounding points of the backward chain
    that is about 8 * 1.1e-3 ~ 1e-2 relative in the worst layer, so this comparison allows 2e-2
    and cosine 0.9998.  The bound of the parity contract (1e-2, 0.9999) applies to the oracle
    that rounds where the kernels do: test_gradients_match_rounded_oracle."""
    import torch
    note("mlp gradients")
    params = fg.mlp_init(5, sub=1)
    sigma = np.array([0.2, 0.3, 0.25])
    m = S.streami_mlp_create(params, sigma, 2 * np.pi)
    rng = np.random.default_rng(4)
    n = 4000
    x = rng.uniform(0, 2 * np.pi, size=(n, 3)).astype(np.float32)
    tgt = (rng.normal(size=(n, 3)) * sigma).astype(np.float32)
    loss, g = S.streami_mlp_train_step(m, torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda(), 0.0,
                                       want_grads=True)
    xhat = omlp.round_bf16(omlp.normalise(x, 2 * np.pi))
    P = bf16_params(params)
    out, cache = omlp.forward(P, xhat, sigma)
    ref = omlp.backward(P, cache, out, tgt.astype(np.float64), sigma)
    assert abs(loss - omlp.loss(out, tgt, sigma)) < 1e-2 * omlp.loss(out, tgt, sigma)
    gl = S.unflatten_params(g)
    for l in range(5):
        for k in range(2):
            a, b = gl[l][k].astype(np.float64), ref[l][k]
            cos = np.sum(a * b) / np.linalg.norm(a) / np.linalg.norm(b)
            assert rel_frob(a, b) < 2e-2 and cos > 0.9998, (l, k, rel_frob(a, b), cos)
    # lr = 0 leaves the parameters untouched
    np.testing.assert_array_equal(S.streami_mlp_get_params(m), S.flatten_params(params))
    S.streami_mlp_destroy(m)


def test_adam_steps_reduce_loss_on_a_fixed_batch(S):
    import torch
    note("mlp training steps")
    params = fg.mlp_init(5, sub=2)
    sigma = np.array([1.0, 1.0, 1.0])
    m = S.streami_mlp_create(params, sigma, 2 * np.pi)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 2 * np.pi, size=(2048, 3)).astype(np.float32)
    tgt = np.stack([np.sin(x[:, 2]), np.cos(x[:, 0]), np.sin(x[:, 1])], 1).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda()
    first, _ = S.streami_mlp_train_step(m, xd, td, 1e-3)
    for _ in range(200):
        last, _ = S.streami_mlp_train_step(m, xd, td, 1e-3, want_loss=False)
    last, _ = S.streami_mlp_train_step(m, xd, td, 1e-3)
    assert last < 0.1 * first, (first, last)
    S.streami_mlp_destroy(m)


def _rounded_oracle(params, x, sigma, period=2 * np.pi):
    """The FP64 network oracle with the matrix cores' rounding points: BF16 weights, input and
    hidden activations (and BF16 gradients entering the backward products)."""
    xhat = omlp.round_bf16(omlp.normalise(x, period))
    P = bf16_params(params)
    out, cache = omlp.forward(P, xhat, sigma, round_act=omlp.round_bf16)
    return P, out, cache


def test_forward_matches_rounded_oracle(S):
    """With the oracle rounding at the same points as the kernel, what is left is FP32
    accumulation order, the fast SiLU and the rare BF16 rounding flip of an activation that
    lies within FP32 noise of a rounding tie; the per-sample error is therefore small against
    the output's own scale."""
    import torch
    note("mlp forward vs rounded oracle")
    params = fg.mlp_init(5, sub=3)
    sigma = np.float32([0.2, 0.3, 0.25]).astype(np.float64)
    m = S.streami_mlp_create(params, sigma, 2 * np.pi)
    rng = np.random.default_rng(6)
    n = 20000
    x = rng.uniform(-7, 13, size=(n, 3)).astype(np.float32)
    out = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    S.streami_mlp_forward(m, torch.from_numpy(x).cuda(), out)
    got = out.cpu().numpy().astype(np.float64)
    _, ref, _ = _rounded_oracle(params, x.astype(np.float64), sigma, float(np.float32(2 * np.pi)))
    err = np.abs(got - ref).max(axis=1) / sigma.max()
    note(f"forward |gpu - rounded oracle| / max sigma: median {np.median(err):.2e} p99 "
         f"{np.quantile(err, 0.99):.2e} max {err.max():.2e}; rel frob {rel_frob(got, ref):.2e}")
    assert rel_frob(got, ref) < 1e-3
    assert np.quantile(err, 0.99) < 1e-3
    S.streami_mlp_destroy(m)


def test_gradients_match_rounded_oracle(S):
    """Gradients of every weight and bias within relative Frobenius 1e-2 and cosine 0.9999 of
    the FP64 oracle that rounds activations and back-propagated gradients to BF16 where the
    kernels do."""
    import torch
    note("mlp gradients vs rounded oracle")
    params = fg.mlp_init(5, sub=1)
    sigma = np.float32([0.2, 0.3, 0.25]).astype(np.float64)
    m = S.streami_mlp_create(params, sigma, 2 * np.pi)
    rng = np.random.default_rng(4)
    n = 4000
    x = rng.uniform(0, 2 * np.pi, size=(n, 3)).astype(np.float32)
    tgt = (rng.normal(size=(n, 3)) * sigma).astype(np.float32)
    loss, g = S.streami_mlp_train_step(m, torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda(), 0.0,
                                       want_grads=True)
    P, out, cache = _rounded_oracle(params, x.astype(np.float64), sigma, float(np.float32(2 * np.pi)))
    ref = omlp.backward(P, cache, out, tgt.astype(np.float64), sigma, round_grad=omlp.round_bf16)
    gl = S.unflatten_params(g)
    worst = []
    for l in range(5):
        for k in range(2):
            a, b = gl[l][k].astype(np.float64), ref[l][k]
            cos = np.sum(a * b) / np.linalg.norm(a) / np.linalg.norm(b)
            worst.append((rel_frob(a, b), cos))
            assert rel_frob(a, b) <= 1e-2 and cos >= 0.9999, (l, k, rel_frob(a, b), cos)
    note("gradient rel frob max %.2e, cosine min %.6f" % (max(w[0] for w in worst), min(w[1] for w in worst)))
    S.streami_mlp_destroy(m)


def test_adam_matches_oracle_over_three_steps(S):
    """k_adam against the oracle's Adam, fed the GPU's own gradients of each step, over three
    steps (bias correction at t = 1, 2, 3): the FP32 master parameters agree to a few FP32
    ulps, so every moment and both bias corrections are those of the definition."""
    import torch
    note("mlp adam vs oracle")
    params = fg.mlp_init(5, sub=4)
    sigma = np.array([0.2, 0.3, 0.25])
    m = S.streami_mlp_create(params, sigma, 2 * np.pi)
    rng = np.random.default_rng(8)
    x = torch.from_numpy(rng.uniform(0, 2 * np.pi, size=(3000, 3)).astype(np.float32)).cuda()
    tgt = torch.from_numpy((rng.normal(size=(3000, 3)) * sigma).astype(np.float32)).cuda()
    lr = 1e-3
    ref = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in params]
    mo, vo = omlp.zeros_like(ref), omlp.zeros_like(ref)
    for t in (1, 2, 3):
        _, g = S.streami_mlp_train_step(m, x, tgt, lr, want_loss=False, want_grads=True)
        gl = [(W.astype(np.float64), b.astype(np.float64)) for W, b in S.unflatten_params(g)]
        omlp.adam_step(ref, gl, mo, vo, t, lr)
        got = S.unflatten_params(S.streami_mlp_get_params(m))
        for l in range(5):
            for k in range(2):
                a, b = got[l][k].astype(np.float64), ref[l][k]
                tol = 4 * np.spacing(np.abs(b).astype(np.float32)).astype(np.float64) + 1e-5 * lr * t
                bad = np.abs(a - b) > tol
                assert not bad.any(), (t, l, k, np.abs(a - b).max())
        # the step moved the parameters (by about lr each)
        assert np.abs(S.flatten_params(got) - S.flatten_params(params)).max() > 0.5 * lr
        ref = [(a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for a, b in ref]
    S.streami_mlp_destroy(m)
