"""Input generator checks: divergence-free turbulence, normalisation, RNE quantisers."""
import numpy as np
import torch

import fieldgen as fg


def test_turbulence_divergence_free_and_normalised():
    # |k| <= 2 on a 28-cell box: wavelengths >= 14 cells, so central differences resolve it
    v = fg.turbulence_values(77, (24, 20, 28), n_modes=64, kmax=2.0)[0]
    assert abs(np.linalg.norm(v, axis=-1).max() - 1.0) < 1e-12
    # central-difference divergence vs gradient magnitude: O(kappa^2 dx^2) relative residue
    div = ((v[1:-1, 1:-1, 2:, 0] - v[1:-1, 1:-1, :-2, 0]) + (v[1:-1, 2:, 1:-1, 1] - v[1:-1, :-2, 1:-1, 1])
           + (v[2:, 1:-1, 1:-1, 2] - v[:-2, 1:-1, 1:-1, 2])) / 2
    grad = np.abs(v[1:-1, 1:-1, 2:, 0] - v[1:-1, 1:-1, :-2, 0]) / 2
    assert np.sqrt(np.mean(div ** 2)) < 0.05 * np.sqrt(np.mean(grad ** 2))


def test_turbulence_slices_drift_and_cache_roundtrip():
    a = fg.turbulence_values(78, (8, 8, 8), n_modes=16, n_slices=3)
    b = fg.turbulence_values(78, (8, 8, 8), n_modes=16, n_slices=3)
    np.testing.assert_array_equal(a, b)
    assert not np.allclose(a[0], a[2])
    assert abs(np.linalg.norm(a, axis=-1).max() - 1.0) < 1e-12


def test_quantizers_round_to_nearest_even():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=20000), rng.normal(size=2000) * 1e-6,
                        [0.5 + 2 ** -12, 0.5 + 3 * 2 ** -12, 65504.0, 65520.0, 1e-9]])
    # FP16: numpy's double -> half conversion is correctly rounded
    np.testing.assert_array_equal(fg.quantize(x, fg.F16).view(np.float16), x.astype(np.float16))
    np.testing.assert_array_equal(fg.quantize(x, fg.F32), x.astype(np.float32))
    # BF16 from values that are exact in FP32 (no double rounding): torch's RNE
    x32 = x.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x32.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(fg.quantize(x32, fg.BF16), ref)


def test_seed_sets():
    s = fg.uniform_seeds(2, 100000, (0, 0, 0), (256, 256, 256))
    assert s.dtype == np.float32 and (s >= 0).all() and (s < 256).all()
    assert abs(s.mean() - 128) < 1.0
    b = fg.blob_seeds(3, 4, 2000, 512.0, 24.0, 8.0)
    assert (b >= 0).all() and (b < 512).all() and b.shape == (8000, 3)
    for k in range(4):
        assert 6.5 < b[k * 2000:(k + 1) * 2000].std(axis=0).mean() < 9.5


def test_turbulence_energy_spectrum_slope():
    """Per-mode amplitudes |k|^-5/6 with |k| uniform in [1, 32] give a shell energy spectrum
    E(k) ~ k^-5/3: a windowed FFT of a 128^3 field recovers the slope over k = 2..24."""
    n = 128
    v = fg.turbulence_values(91, (n, n, n), n_modes=512, kmin=1.0, kmax=32.0)[0][1:-1, 1:-1, 1:-1]
    w = np.hanning(n)
    win = w[:, None, None] * w[None, :, None] * w[None, None, :]
    k = np.fft.fftfreq(n) * n
    shell = np.rint(np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)).astype(int)
    energy = np.zeros(n)
    for c in range(3):
        power = np.abs(np.fft.fftn(v[..., c] * win)) ** 2
        energy += np.bincount(shell.ravel(), weights=power.ravel(), minlength=n)[:n]
    ks = np.arange(2, 25)
    slope = np.polyfit(np.log(ks), np.log(energy[ks]), 1)[0]
    assert abs(slope + 5.0 / 3.0) < 0.2, slope


def test_partition_samples_the_whole_field():
    """Each sub-block of a partition interpolates the same field as the whole block wherever
    its sample domain reaches (its ghost layer is the neighbours' nodes), including the
    strip of the halo beyond its owned bounds; bounds tile the whole block."""
    import oracle
    whole = fg.turbulence_block(2, edge=12, dims=(12, 8, 16), rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
    parts = fg.partition(whole, (3, 2, 2))
    W = oracle.Field.from_block(whole)
    rng = np.random.default_rng(0)
    vol = 0.0
    for p in parts:
        P = oracle.Field.from_block(p)
        lo, hi = np.array(p.lo) - 0.5, np.array(p.hi) + 0.5  # owned bounds + the half-cell halo
        x = rng.uniform(lo, hi, size=(500, 3))
        vw, okw = W.sample(x)
        vp, okp = P.sample(x)
        assert okp.all()
        np.testing.assert_allclose(vp[okw], vw[okw], rtol=0, atol=1e-12)
        vol += np.prod(np.array(p.hi) - np.array(p.lo))
        assert p.rank_grid == (3, 2, 2)
    assert vol == 12 * 8 * 16


def _near_tie(values, fmt):
    """True where an FP64 value lies within 1e-12 (relative) of a rounding tie of fmt: two
    correct evaluations of the same sum may then round to different stored values."""
    mant = {fg.F16: 10, fg.BF16: 7}[fmt]
    emin = {fg.F16: -14, fg.BF16: -126}[fmt]
    _, e = np.frexp(values)
    ulp = np.ldexp(1.0, np.maximum(e - 1, emin) - mant)
    frac = np.abs(values / ulp - np.floor(values / ulp) - 0.5)
    return frac * ulp <= 1e-12 * np.maximum(np.abs(values), 1e-300)


def test_rne_torch_matches_host_quantiser():
    from fieldgen import device as fgd
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.normal(size=50000), rng.normal(size=5000) * 1e-6, rng.normal(size=2000) * 1e-9,
                        [0.0, -0.0, 0.5 + 2 ** -12, 0.5 + 3 * 2 ** -12, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 65504.0]])
    t = torch.from_numpy(x)
    for fmt in (fg.F16, fg.BF16):
        got = fgd.rne_torch(t, fmt).numpy().view(np.uint16)
        np.testing.assert_array_equal(got, fg.quantize(x, fmt))
    np.testing.assert_array_equal(fgd.rne_torch(t, fg.F32).numpy(), fg.quantize(x, fg.F32))


def test_device_turbulence_equals_host_turbulence():
    """The torch generator (run here on the CPU) gives the host generator's field: FP64 values
    within summation-order rounding, stored values identical except at rounding ties."""
    from fieldgen import device as fgd
    dims, S = (21, 17, 26), 3
    ref = fg.turbulence_values(79, dims, sub=2, n_modes=48, n_slices=S)
    for fmt in (fg.F16, fg.BF16):
        stored, vals = fgd.turbulence_stored(79, dims, sub=2, n_modes=48, n_slices=S, fmt=fmt, device="cpu",
                                             want_values=True)
        assert stored.shape == (S, dims[2] + 2, dims[1] + 2, dims[0] + 2, 3)
        np.testing.assert_allclose(vals.numpy(), ref, rtol=0, atol=1e-13)
        got = stored.numpy().view(np.uint16)
        want = fg.quantize(ref, fmt)
        differ = got != want
        assert not (differ & ~_near_tie(ref, fmt)).any()
        assert differ.mean() < 1e-4


def test_device_streakline_particles_equal_host_ones():
    from fieldgen import device as fgd
    em = fg.uniform_seeds(4, 300, (0, 0, 0), (40, 50, 60), sub=7)
    lim = fg.int_uniform(4, fg.P_MAXSTEPS, 300, 1, 95, sub=3).astype(np.int32)
    ref = fg.streakline_particles(em, lim, 10, 0.5)
    got = fgd.streakline_particles(torch.from_numpy(em), torch.from_numpy(lim), 10, 0.5)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a.numpy(), b)
