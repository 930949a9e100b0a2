"""Brute-force references for tiny inputs -- TEST INFRASTRUCTURE ONLY.

  dft(y)          O(N^2) discrete Fourier transform, exp(-2 pi i k n / N)
  xf_frame(a, b)  lag-domain (XF) correlation of one frame folded to N lags
                  and Fourier transformed with dft(); equals A[k] conj(B[k])
                  exactly (convolution theorem), so it checks FX without
                  sharing its transform.
"""
from __future__ import annotations

import numpy as np


def dft(y: np.ndarray) -> np.ndarray:
    """Plain O(N^2) DFT along the last axis, rows of the matrix built per block of k."""
    y = np.asarray(y, dtype=np.complex128)
    N = y.shape[-1]
    n = np.arange(N, dtype=np.int64)
    out = np.empty(y.shape, dtype=np.complex128)
    for k0 in range(0, N, 256):
        k = np.arange(k0, min(N, k0 + 256), dtype=np.int64)
        # reduce k*n modulo N in integers so the angle is exact before scaling
        ang = -2.0 * np.pi * ((k[:, None] * n[None, :]) % N) / N
        out[..., k0:k0 + k.shape[0]] = y @ np.exp(1j * ang).T
    return out


def lag_correlation(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """lin[m + N - 1] = sum_n a[n + m] conj(b[n]) for -N < m < N (one frame)."""
    N = a.shape[0]
    lin = np.zeros(2 * N - 1, dtype=np.complex128)
    for m in range(-(N - 1), N):
        lo, hi = max(0, -m), min(N, N - m)
        lin[m + N - 1] = np.sum(a[lo + m:hi + m] * np.conj(b[lo:hi]))
    return lin


def xf_frame(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Cross power spectrum of one frame via the lag domain (all N bins)."""
    N = a.shape[0]
    lin = lag_correlation(a, b)
    c = np.zeros(N, dtype=np.complex128)
    for m in range(-(N - 1), N):
        c[m % N] += lin[m + N - 1]        # fold lag m and m - N onto one circular lag
    return dft(c)
