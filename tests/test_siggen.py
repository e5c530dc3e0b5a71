"""The seeded input generators (no method arithmetic): the device-side
synthesis draws what the numpy path draws and meets the stated SNR."""
import numpy as np
import pytest

import siggen

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("N,s", [(4096, 8), (3 * 2 ** 12 + 1, 40)])
def test_device_synthesis_matches_numpy_path(N, s):
    ref = siggen.sparse_signal(N, s, seed=11)
    f, freqs, coefs = siggen.sparse_signal_device(N, s, seed=11, snr_db=None, device="cpu")
    assert np.array_equal(freqs, ref.freqs) and np.array_equal(coefs, ref.coefs)
    assert f.dtype == torch.complex64
    assert np.max(np.abs(f.numpy() - ref.f32)) <= 1e-5 * np.max(np.abs(ref.f))


def test_device_noise_is_exact_snr_and_seeded():
    N, s, snr = 8192, 16, 25.0
    clean = siggen.sparse_signal_device(N, s, seed=3, snr_db=None, device="cpu")[0].numpy().astype(np.complex128)
    a = siggen.sparse_signal_device(N, s, seed=3, snr_db=snr, device="cpu")[0].numpy().astype(np.complex128)
    b = siggen.sparse_signal_device(N, s, seed=3, snr_db=snr, device="cpu")[0].numpy()
    assert np.array_equal(a.astype(np.complex64), b)
    got = 20 * np.log10(np.linalg.norm(clean) / np.linalg.norm(a - clean))
    assert abs(got - snr) < 1e-3


def test_batched_shapes_cover_the_stated_lengths():
    shapes = siggen.batched_shapes(0)
    assert len(shapes) == 256
    assert {n for n, _, _ in shapes} <= set(siggen.BATCHED_LENGTHS)
    assert all(16 <= s <= 256 for _, s, _ in shapes)
