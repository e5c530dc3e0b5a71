"""Seeded synthetic inputs for the sparse Fourier transform.

This module only *draws* inputs; it holds none of the transform's arithmetic.
Both the FP64 oracle (under ``oracle/``) and the GPU library are fed from here,
and neither imports the other.

Conventions (shared by every workload):

* frequency band ``B = (-ceil(N/2), floor(N/2)]`` (Section 2, definition of B);
* coefficients ``c_w`` with ``f_j = sum_w c_w exp(2 pi i w j / N)``, i.e.
  ``c_w = numpy.fft.fft(f)[w mod N] / N``.  The paper samples at
  ``-pi + 2 pi j / N`` and so its ``fhat_w`` equals ``(-1)^w c_w``;
* signal generator of the experiments (Section 5.1): ``s`` distinct
  frequencies drawn uniformly from ``B``, unit-magnitude coefficients with
  uniform phase, ``f`` formed by an inverse DFT;
* noise of Section 5.4: i.i.d. complex Gaussian entries (real and imaginary
  parts standard normal), rescaled so that ``20 log10(||f|| / ||n||)`` equals
  the requested SNR exactly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "band_limits", "SparseSignal", "draw_frequencies", "draw_coefficients",
    "synthesize", "add_noise", "sparse_signal", "workload",
    "WORKLOADS", "batched_shapes", "serving_requests", "sparse_signal_device",
]


def band_limits(N: int) -> tuple[int, int]:
    """Smallest and largest frequency of B = (-ceil(N/2), floor(N/2)]."""
    return -((N + 1) // 2) + 1, N // 2


@dataclasses.dataclass
class SparseSignal:
    N: int
    s: int
    freqs: np.ndarray          # int64, in B, draw order
    coefs: np.ndarray          # complex128
    snr_db: Optional[float]    # None = noiseless
    f: np.ndarray              # complex128 samples f_j (noise included)
    f_clean: np.ndarray        # complex128 samples without noise

    @property
    def f32(self) -> np.ndarray:
        """The complex64 rounding of f, which is what both sides consume."""
        return self.f.astype(np.complex64)


def draw_frequencies(N: int, s: int, rng: np.random.Generator) -> np.ndarray:
    lo, _ = band_limits(N)
    picks = rng.choice(N, size=s, replace=False)
    return (picks.astype(np.int64) + lo)


def draw_coefficients(s: int, rng: np.random.Generator, magnitude: str = "unit") -> np.ndarray:
    phase = np.exp(2j * np.pi * rng.random(s))
    if magnitude == "unit":
        mag = np.ones(s)
    elif magnitude == "loguniform":
        mag = 10.0 ** rng.uniform(-2.0, 0.0, size=s)
    else:
        raise ValueError(magnitude)
    return mag * phase


def synthesize(N: int, freqs: np.ndarray, coefs: np.ndarray) -> np.ndarray:
    """f_j = sum_w c_w exp(2 pi i w j / N), j = 0..N-1, in complex128."""
    spec = np.zeros(N, dtype=np.complex128)
    np.add.at(spec, np.mod(freqs, N), coefs)
    return np.fft.ifft(spec) * N


def add_noise(f: np.ndarray, snr_db: float, rng: np.random.Generator) -> np.ndarray:
    n = rng.standard_normal(f.shape[0]) + 1j * rng.standard_normal(f.shape[0])
    scale = np.linalg.norm(f) / (np.linalg.norm(n) * 10.0 ** (snr_db / 20.0))
    return f + scale * n


def sparse_signal(N: int, s: int, seed: int, snr_db: Optional[float] = None,
                  magnitude: str = "unit") -> SparseSignal:
    rng = np.random.Generator(np.random.PCG64(seed))
    freqs = draw_frequencies(N, s, rng)
    coefs = draw_coefficients(s, rng, magnitude)
    f_clean = synthesize(N, freqs, coefs)
    f = f_clean if snr_db is None else add_noise(f_clean, snr_db, rng)
    return SparseSignal(N, s, freqs, coefs, snr_db, f, f_clean)


def sparse_signal_device(N: int, s: int, seed: int, snr_db: Optional[float] = None,
                         magnitude: str = "unit", device: str = "cuda"):
    """The generator of sparse_signal with the synthesis and the noise on a
    torch device (for large batches): the same frequencies and coefficients
    (numpy PCG64(seed)), f = N ifft(c) in complex128 on the device, noise from
    torch's generator seeded with `seed` (so it differs from sparse_signal's
    noise), rescaled to the exact SNR.  Returns (f complex64 tensor, freqs, coefs)."""
    import torch

    rng = np.random.Generator(np.random.PCG64(seed))
    freqs = draw_frequencies(N, s, rng)
    coefs = draw_coefficients(s, rng, magnitude)
    spec = torch.zeros(N, dtype=torch.complex128, device=device)
    spec.index_put_((torch.from_numpy(np.mod(freqs, N)).to(device),),
                    torch.from_numpy(coefs).to(device), accumulate=True)
    f = torch.fft.ifft(spec) * N
    if snr_db is not None:
        g = torch.Generator(device=device)
        g.manual_seed(seed)
        n = torch.complex(torch.randn(N, dtype=torch.float64, device=device, generator=g),
                          torch.randn(N, dtype=torch.float64, device=device, generator=g))
        f = f + n * (torch.linalg.vector_norm(f) / (torch.linalg.vector_norm(n) * 10.0 ** (snr_db / 20.0)))
    return f.to(torch.complex64), freqs, coefs


# The five workloads.  Keys name what they are.
WORKLOADS = {
    # one signal, exactness: N=2^14, s=8, noiseless, complex128 original
    "plain_n2e14_s8": dict(N=2 ** 14, s=8, snr_db=None, magnitude="unit"),
    # headline GPU shape: N=2^22, s=64, 20 dB
    "plain_n2e22_s64_20db": dict(N=2 ** 22, s=64, snr_db=20.0, magnitude="unit"),
    # prime length: N=10,000,019, s=128, log-uniform magnitudes, 40 dB
    "prime_n10000019_s128_40db": dict(N=10_000_019, s=128, snr_db=40.0, magnitude="loguniform"),
}


def workload(name: str, seed: int) -> SparseSignal:
    w = WORKLOADS[name]
    return sparse_signal(w["N"], w["s"], seed, w["snr_db"], w["magnitude"])


BATCHED_LENGTHS = [2 ** k for k in range(18, 25)] + [3 * 2 ** 20, 5 * 2 ** 19 + 1]


def batched_shapes(batch_seed: int, count: int = 256) -> list[tuple[int, int, int]]:
    """(N, s, signal seed) for the uneven batch: N uniform over 2^18..2^24,
    3*2^20 and 5*2^19+1; s uniform integer in [16, 256]; 30 dB noise."""
    rng = np.random.Generator(np.random.PCG64(10_000 + batch_seed))
    out = []
    for i in range(count):
        N = int(BATCHED_LENGTHS[rng.integers(len(BATCHED_LENGTHS))])
        s = int(rng.integers(16, 257))
        out.append((N, s, 1_000_000 * (batch_seed + 1) + i))
    return out


def serving_requests(seed: int, count: int, rate_hz: float,
                     min_log2: int = 20, max_log2: int = 26) -> list[dict]:
    """Poisson arrivals; N uniform over 2^min_log2..2^max_log2; s log-uniform in
    [16, 1024]; SNR uniform in [0, 40] dB; unit-magnitude coefficients."""
    rng = np.random.Generator(np.random.PCG64(20_000 + seed))
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        N = 2 ** int(rng.integers(min_log2, max_log2 + 1))
        s = int(round(math.exp(rng.uniform(math.log(16), math.log(1024)))))
        snr = float(rng.uniform(0.0, 40.0))
        out.append(dict(t=t, N=N, s=s, snr_db=snr, seed=2_000_000 + 7919 * seed + i))
    return out
