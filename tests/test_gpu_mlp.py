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
