"""GPU tests of the learned flow-map surrogate form.

The network's own accuracy is learned (parity unpinned); what is pinned:
  * the training windows equal the FP64 oracle's 16-step flow map;
  * with tolerance 0 every jump is rejected and the surrogate mode must be
    bit-identical to plain RK4 (the fallback is the plain integrator);
  * with an infinite tolerance every jump is the network displacement;
  * after training, the network's endpoint error is reported against the
    plain-RK4 oracle together with the acceptance rate.
"""
import sys

import numpy as np
import pytest

import fieldgen as fg
import oracle

pytestmark = pytest.mark.gpu

H = 0.01


def note(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_02627_amd as S
    S._load()
    return S


@pytest.fixture(scope="module")
def trained(S):
    import torch
    from paper_2606_02627_amd import surrogate
    note("surrogate: training windows + short training")
    blk = fg.abc_block(32)
    starts = fg.training_starts(5, 1 << 18, 2 * np.pi)
    x0, d = surrogate.flow_map_windows(blk, starts, H)
    net, sigma, hist = surrogate.train(x0, d, fg.mlp_init(5), 2 * np.pi, epochs=12, batch=8192, lr=2e-3)
    yield blk, starts, x0, d, net, sigma, hist
    S.streami_mlp_destroy(net)


def test_training_windows_match_oracle(S, trained):
    blk, starts, x0, d, *_ = trained
    F = oracle.Field.from_block(blk)
    k = 4096
    ref = F.trace(starts[:k], float(np.float32(H)), 16)
    got = x0[:k].cpu().numpy().astype(np.float64) + d[:k].cpu().numpy().astype(np.float64)
    assert np.abs(got - ref["final_pos"]).max() < 1e-4 * 2 * np.pi
    np.testing.assert_array_equal(x0[:k].cpu().numpy(), starts[:k])


def test_training_reduces_loss(trained):
    hist = trained[6]
    note("training loss per epoch:", [round(h["loss"], 5) for h in hist])
    assert hist[-1]["loss"] < 0.1 * hist[0]["loss"] and hist[-1]["loss"] < 0.1, hist


def _run(S, blk, seeds, steps, **kw):
    f = S.Field([blk], S.F32)
    f.seed(0, seeds, default_max_steps=steps, record_stride=16)
    st = f.advect(H, **kw)
    L = f.lines(0)
    f.close()
    return st, L


def test_tolerance_zero_is_plain_rk4_bit_exact(S, trained):
    blk, net = trained[0], trained[4]
    note("surrogate tol=0 vs plain")
    seeds = fg.uniform_seeds(5, 3000, (0, 0, 0), (2 * np.pi,) * 3, sub=11)
    st_p, Lp = _run(S, blk, seeds, 200)
    for kind in (0, 1):
        st_s, Ls = _run(S, blk, seeds, 200, mode=S.MODE_SURROGATE, mlp=net, residual_tol_cells=0.0,
                        residual_kind=kind)
        assert st_s.surrogate_accepted == 0 and st_s.steps == st_p.steps
        for k in ("offsets", "xyz", "steps", "codes"):
            np.testing.assert_array_equal(Ls[k], Lp[k])


def test_infinite_tolerance_takes_network_jumps(S, trained):
    import torch
    from paper_2606_02627_amd import surrogate
    blk, net = trained[0], trained[4]
    note("surrogate tol=inf")
    seeds = fg.uniform_seeds(5, 1000, (0, 0, 0), (2 * np.pi,) * 3, sub=12)
    st, L = _run(S, blk, seeds, 16, mode=S.MODE_SURROGATE, mlp=net, residual_tol_cells=3e38, residual_kind=1)
    assert st.surrogate_accepted == 1000 and st.surrogate_fallback == 0
    dnet = surrogate.predict(net, torch.from_numpy(seeds).cuda()).cpu().numpy()
    got = L["xyz"].reshape(1000, 2, 3)[:, 1]
    np.testing.assert_array_equal(got, (seeds + dnet).astype(np.float32))


def test_trained_surrogate_endpoint_error_and_acceptance(S, trained):
    blk, net = trained[0], trained[4]
    note("surrogate endpoint error")
    seeds = fg.uniform_seeds(5, 4096, (0, 0, 0), (2 * np.pi,) * 3, sub=13)
    steps = 400
    ref = oracle.Field.from_block(blk).trace(seeds, float(np.float32(H)), steps, keep_verts=False)
    ext = 2 * np.pi
    for kind in (0, 1):
        st, L = _run(S, blk, seeds, steps, mode=S.MODE_SURROGATE, mlp=net, residual_tol_cells=1e-3,
                     residual_kind=kind)
        assert st.steps == 4096 * steps and (L["steps"] == steps).all()
        end = L["xyz"][L["offsets"][1:] - 1].astype(np.float64)
        err = np.abs(end - ref["final_pos"]).max(axis=1) / ext
        acc = st.surrogate_accepted / max(1, st.surrogate_accepted + st.surrogate_fallback)
        note(f"kind {kind}: acceptance {acc:.3f}, endpoint error / extent median {np.median(err):.2e} "
             f"p90 {np.quantile(err, 0.9):.2e} max {err.max():.2e}")
        assert np.isfinite(err).all()


def test_full_size_properties(S, trained):
    """The surrogate workload's size and launch: 2^22 ABC seeds, 2000 steps (125 jumps), every
    16th vertex kept.  Tolerance 0 reproduces plain RK4 exactly (step and termination counts of
    all particles, the lines of a sampled range); an infinite tolerance takes every jump, and the
    sampled range ends at the network displacement applied 125 times."""
    import torch
    from paper_2606_02627_amd import surrogate
    blk, net = trained[0], trained[4]
    n, first, count = 1 << 22, 777, 4096
    note("surrogate full size")
    d_seeds = torch.from_numpy(fg.uniform_seeds(5, n, (0, 0, 0), (2 * np.pi,) * 3, sub=21)).cuda()

    def run(**kw):
        f = S.Field([blk], S.F32)
        f.seed(0, d_seeds, default_max_steps=2000, record_stride=16)
        st = f.advect(H, **kw)
        L = f.lines(0, first, count)
        f.close()
        return st, L

    st_p, Lp = run()
    st_0, L0 = run(mode=S.MODE_SURROGATE, mlp=net, residual_tol_cells=0.0, residual_kind=1)
    assert st_0.surrogate_accepted == 0 and st_0.steps == st_p.steps == n * 2000
    assert list(st_0.terminated) == list(st_p.terminated)
    for k in ("offsets", "xyz", "steps", "codes", "ids"):
        np.testing.assert_array_equal(L0[k], Lp[k])
    st_i, Li = run(mode=S.MODE_SURROGATE, mlp=net, residual_tol_cells=3e38, residual_kind=1)
    assert st_i.surrogate_accepted == n * 125 and st_i.surrogate_fallback == 0
    x = d_seeds[first:first + count].clone()
    for _ in range(125):
        x = x + surrogate.predict(net, x)
    np.testing.assert_array_equal(Li["xyz"][Li["offsets"][1:] - 1], x.cpu().numpy())
