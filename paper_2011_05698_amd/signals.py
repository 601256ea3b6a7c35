"""Seeded synthetic test signals (the experimental setup of Sec. 4.1).

K frequencies drawn uniformly without replacement from [0, N), each with
magnitude 1 (or log-uniform magnitudes) and a uniform random phase; the time
signal is the inverse DFT in the paper's normalisation (Eq. 2: the forward
transform carries 1/N, so x_j = sum_f xhat_f exp(+2 pi i f j / N)), optionally
plus complex white Gaussian noise at a given SNR.

This module holds no part of the sparse-FFT method.  Both the product path
and the CPU checker receive the signals it produces.
"""

from __future__ import annotations

import numpy as np

__all__ = ["planted_spectrum", "time_signal", "add_noise", "SignalSpec", "make_signal"]


def planted_spectrum(N: int, K: int, seed: int, mags: str = "unit", mag_range=(1e-2, 1.0)):
    """Sorted support (int64) and complex128 values of a K-sparse spectrum."""
    rng = np.random.default_rng(seed)
    support = np.sort(rng.choice(N, size=K, replace=False)).astype(np.int64)
    if mags == "unit":
        amp = np.ones(K)
    elif mags == "loguniform":
        lo, hi = np.log(mag_range[0]), np.log(mag_range[1])
        amp = np.exp(rng.uniform(lo, hi, size=K))
    else:
        raise ValueError(f"unknown magnitude law {mags!r}")
    phase = rng.uniform(0.0, 2.0 * np.pi, size=K)
    return support, amp * np.exp(1j * phase)


def time_signal(N: int, support, values) -> np.ndarray:
    """x = N * ifft(xhat): the time signal whose Eq. 2 spectrum is xhat."""
    xhat = np.zeros(N, dtype=np.complex128)
    xhat[np.asarray(support)] = values
    return np.fft.ifft(xhat) * N


def add_noise(x: np.ndarray, snr_db: float, seed: int) -> np.ndarray:
    """Add circular complex Gaussian noise CN(0, s^2) with
    s^2 = (||x||^2 / N) 10^(-snr/10) (total-energy SNR)."""
    rng = np.random.default_rng(seed)
    N = x.shape[0]
    s2 = float(np.vdot(x, x).real) / N * 10.0 ** (-snr_db / 10.0)
    noise = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return x + noise * np.sqrt(s2 / 2.0)


class SignalSpec:
    """A reproducible test signal: N, K, seed, optional SNR and magnitude law."""

    def __init__(self, N, K, seed, snr_db=None, mags="unit"):
        self.N, self.K, self.seed, self.snr_db, self.mags = N, K, seed, snr_db, mags

    def __repr__(self):
        return f"SignalSpec(N={self.N}, K={self.K}, seed={self.seed}, snr_db={self.snr_db}, mags={self.mags!r})"


def make_signal(spec: SignalSpec):
    """(x complex128, support, values) for a SignalSpec."""
    support, values = planted_spectrum(spec.N, spec.K, spec.seed, spec.mags)
    x = time_signal(spec.N, support, values)
    if spec.snr_db is not None:
        x = add_noise(x, spec.snr_db, spec.seed + 0x5EED)
    return x, support, values
