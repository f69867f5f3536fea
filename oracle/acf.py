"""Autocovariance estimates of a stretch of strain (Sec. II.B item 6): direct correlation
of the data, or a Welch PSD followed by its inverse Fourier transform, truncated to the
lags a segment needs.  Plain FP64 NumPy, test infrastructure only.

direct : acf[k] = (1/n) sum_{t < n-k} x_t x_{t+k}   (biased sample autocovariance)
welch  : segments of length L with half overlap, mean removed, periodic Hann window w;
         two-sided density periodogram P_s[f] = |DFT(w y_s)[f]|^2 / (fs sum w^2),
         averaged over segments (mean); acf = fs * IDFT(P)[:n_lags].
"""
from __future__ import annotations

import numpy as np


def acf_direct(x: np.ndarray, n_lags: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    return np.array([np.dot(x[:n - k], x[k:]) / n for k in range(n_lags)])


def hann_periodic(L: int) -> np.ndarray:
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * np.arange(L) / L)


def welch_psd_two_sided(x: np.ndarray, L: int, fs: float = 1.0) -> np.ndarray:
    """Mean-averaged Welch periodogram, two-sided, density scaling."""
    x = np.asarray(x, dtype=np.float64)
    w = hann_periodic(L)
    starts = range(0, len(x) - L + 1, L // 2)
    P = np.zeros(L)
    K = 0
    for s in starts:
        seg = x[s:s + L]
        X = np.fft.fft(w * (seg - seg.mean()))
        P += np.abs(X) ** 2 / (fs * np.sum(w * w))
        K += 1
    return P / K


def acf_welch(x: np.ndarray, L: int, n_lags: int, fs: float = 1.0) -> np.ndarray:
    P = welch_psd_two_sided(x, L, fs)
    return (fs * np.fft.ifft(P).real)[:n_lags]
