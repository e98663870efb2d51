"""The allocation-free training step (streami_mlp_train_step_noalloc) against the allocating
one (streami_mlp_train_step), through the C-ABI, on the GPU.

Both run the same kernels on the same inputs, so gradients and updated parameters must be
bit-identical; the batch loss is summed with atomics in an unspecified order, so it agrees to
FP32 rounding.  Two calls in a row, the second with a smaller batch that is not a multiple of
the 32-row padding, check that the static workspace's leftovers from the first call do not
leak into the second."""
import sys

import numpy as np
import pytest

import fieldgen as fg

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def _batch(n, sub):
    import torch
    x = fg.training_starts(5, n, 2 * np.pi, sub=sub).astype(np.float32)
    t = (0.05 * np.sin(x[:, [1, 2, 0]]) + 0.02 * np.cos(x)).astype(np.float32)  # any smooth target
    return torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()


def test_noalloc_train_step_matches_train_step():
    import torch
    import paper_2606_02627_amd as S
    S._load()
    assert torch.cuda.is_available()
    init, sigma, period = fg.mlp_init(5), np.array([0.05, 0.06, 0.07]), 2 * np.pi
    a = S.streami_mlp_create(init, sigma, period)
    b = S.streami_mlp_create(init, sigma, period)
    try:
        for call, (n, lr) in enumerate(((S.MLP_NOALLOC_MAX_BATCH, 1e-3), (1000, 2e-3))):
            note(f"no-alloc training step: call {call}, batch {n}, lr {lr}")
            x, t = _batch(n, sub=40 + call)
            la, ga = S.streami_mlp_train_step(a, x, t, lr, want_loss=True, want_grads=True)
            lb, gb = S.streami_mlp_train_step_noalloc(b, x, t, lr, want_loss=True, want_grads=True)
            assert np.isfinite(la) and la > 0
            assert abs(la - lb) <= 1e-5 * la, (la, lb)
            np.testing.assert_array_equal(ga, gb)
            pa, pb = S.streami_mlp_get_params(a), S.streami_mlp_get_params(b)
            np.testing.assert_array_equal(pa, pb)
            assert not np.array_equal(pa, S.flatten_params(init))  # the step did update the weights
            oa, ob = torch.zeros_like(x), torch.zeros_like(x)
            S.streami_mlp_forward(a, x, oa)
            S.streami_mlp_forward(b, x, ob)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(oa.cpu().numpy(), ob.cpu().numpy())
        # a batch beyond the static workspace is refused before any device work; the handle stays usable
        x, t = _batch(S.MLP_NOALLOC_MAX_BATCH + 1, sub=50)
        with pytest.raises(S.StreamiError, match="allocation-free"):
            S.streami_mlp_train_step_noalloc(b, x, t, 1e-3)
        x, t = _batch(64, sub=51)
        lb, _ = S.streami_mlp_train_step_noalloc(b, x, t, 0.0)
        la, _ = S.streami_mlp_train_step(a, x, t, 0.0)
        assert abs(la - lb) <= 1e-5 * la
    finally:
        S.streami_mlp_destroy(a)
        S.streami_mlp_destroy(b)
