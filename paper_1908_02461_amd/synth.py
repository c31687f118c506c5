"""Seeded synthetic inputs: planted k-sparse spectra plus complex Gaussian noise.

This module builds inputs only; it holds none of the sparse-FFT method's
arithmetic.  Both the GPU tests and the oracle tests draw their inputs here.

The workload follows the paper's experiments (Sec. IV): k frequencies chosen
at random, the rest zero.  The time signal is the inverse DFT of the planted
spectrum, x_u = (1/n) sum_f a_f e^{+2 pi i f u / n}, so that the unnormalised
forward DFT of x returns a_f exactly.  Noise is circular complex Gaussian
with per-sample variance mean|x|^2 / 10^(SNR/10); by Parseval the same ratio
holds in the frequency domain.
"""
from __future__ import annotations

import numpy as np


def _magnitudes(rng: np.random.Generator, k: int, mag) -> np.ndarray:
    if mag is None or mag == 1.0 or mag == "one":
        return np.ones(k)
    kind, lo, hi = mag
    if kind == "uniform":
        return rng.uniform(lo, hi, size=k)
    if kind == "loguniform":
        return np.exp(rng.uniform(np.log(lo), np.log(hi), size=k))
    raise ValueError(f"unknown magnitude law {kind!r}")


def _noise(rng: np.random.Generator, x: np.ndarray, snr_db) -> np.ndarray:
    if snr_db is None:
        return x
    p_sig = float(np.mean(np.abs(x) ** 2))
    var = p_sig / (10.0 ** (snr_db / 10.0))
    scale = np.sqrt(var / 2.0)
    noise = rng.standard_normal(x.shape) * scale + 1j * rng.standard_normal(x.shape) * scale
    return x + noise


def planted_1d(n: int, k: int, seed: int, mag=None, snr_db=None, dtype=np.complex128):
    """Return (x, locs ascending, amplitudes at locs) for a length-n signal."""
    rng = np.random.Generator(np.random.PCG64(seed))
    locs = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
    amps = _magnitudes(rng, k, mag) * np.exp(1j * rng.uniform(0.0, 2 * np.pi, size=k))
    X = np.zeros(n, dtype=np.complex128)
    X[locs] = amps
    x = np.fft.ifft(X)
    x = _noise(rng, x, snr_db)
    return x.astype(dtype), locs, amps


def planted_2d(N: int, k: int, seed: int, mag=None, snr_db=None, dtype=np.complex128):
    """Return (x [N,N], linear locs f1*N+f2 ascending, amplitudes) for an N x N image."""
    rng = np.random.Generator(np.random.PCG64(seed))
    locs = np.sort(rng.choice(N * N, size=k, replace=False)).astype(np.int64)
    amps = _magnitudes(rng, k, mag) * np.exp(1j * rng.uniform(0.0, 2 * np.pi, size=k))
    X = np.zeros(N * N, dtype=np.complex128)
    X[locs] = amps
    x = np.fft.ifft2(X.reshape(N, N))
    x = _noise(rng, x, snr_db)
    return x.astype(dtype), locs, amps


# The workloads, by name, with their sizes (sizes and distributions of the
# paper's synthetic experiments, widened to the 1D and noisy cases).
WORKLOADS = {
    "c1_1d_c128_n16k_k8": dict(ndim=1, n=1 << 14, k=8, mag=None, snr_db=None, dtype="c128"),
    "c2_1d_c64_n4m_k64_snr40": dict(ndim=1, n=1 << 22, k=64, mag=("uniform", 0.5, 1.0), snr_db=40.0,
                                    dtype="c64"),
    "c3_2d_c64_n4096_k256_snr30": dict(ndim=2, n=4096, k=256, mag=("loguniform", 0.1, 1.0),
                                       snr_db=30.0, dtype="c64"),
}


def make(workload: str, seed: int):
    w = WORKLOADS[workload]
    dt = np.complex64 if w["dtype"] == "c64" else np.complex128
    fn = planted_1d if w["ndim"] == 1 else planted_2d
    return fn(w["n"], w["k"], seed, mag=w["mag"], snr_db=w["snr_db"], dtype=dt)


def planted_1d_device(n: int, k: int, seed: int, mag=None, snr_db=None, device="cuda"):
    """planted_1d built on the GPU (complex64) for large benchmark batches:
    the same recipe, with the inverse DFT and the noise drawn by torch."""
    import torch

    rng = np.random.Generator(np.random.PCG64(seed))
    locs = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
    amps = _magnitudes(rng, k, mag) * np.exp(1j * rng.uniform(0.0, 2 * np.pi, size=k))
    X = torch.zeros(n, dtype=torch.complex64, device=device)
    X[torch.from_numpy(locs).to(device)] = torch.from_numpy(amps.astype(np.complex64)).to(device)
    x = torch.fft.ifft(X)
    if snr_db is not None:
        g = torch.Generator(device=device)
        g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
        p_sig = float(torch.mean(torch.abs(x) ** 2))
        scale = float(np.sqrt(p_sig / (10.0 ** (snr_db / 10.0)) / 2.0))
        noise = torch.randn(n, generator=g, device=device) + 1j * torch.randn(n, generator=g, device=device)
        x = x + (noise * scale).to(torch.complex64)
    return x, locs, amps


def planted_2d_device(N: int, k: int, seed: int, mag=None, snr_db=None, device="cuda"):
    """planted_2d built on the GPU (complex64): the same recipe, with the
    inverse DFT and the noise drawn by torch."""
    import torch

    rng = np.random.Generator(np.random.PCG64(seed))
    locs = np.sort(rng.choice(N * N, size=k, replace=False)).astype(np.int64)
    amps = _magnitudes(rng, k, mag) * np.exp(1j * rng.uniform(0.0, 2 * np.pi, size=k))
    X = torch.zeros(N * N, dtype=torch.complex64, device=device)
    X[torch.from_numpy(locs).to(device)] = torch.from_numpy(amps.astype(np.complex64)).to(device)
    x = torch.fft.ifft2(X.view(N, N))
    del X
    if snr_db is not None:
        g = torch.Generator(device=device)
        g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
        p_sig = float(torch.mean(torch.abs(x) ** 2))
        scale = float(np.sqrt(p_sig / (10.0 ** (snr_db / 10.0)) / 2.0))
        x = x + (torch.randn(N, N, generator=g, device=device)
                 + 1j * torch.randn(N, N, generator=g, device=device)).to(torch.complex64) * scale
    return x, locs, amps
