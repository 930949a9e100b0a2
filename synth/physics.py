"""Exact-physics station voltages for a small number of stations.

Forward model (what an antenna records; no correlator arithmetic):

  * the sky emits a real white Gaussian signal s(t), sampled on the reference
    (geocentric) time grid k/fs; its analytic companion is s + i H{s};
  * the wavefront reaches station s at station time t_st = t + tau_true(t),
    tau_true = model polynomial + a constant residual delta (the part the
    correlator's model does not know);
  * after mixing down with a fixed LO at nu0 (upper sideband), the real
    baseband sample at station time t_st is
        x = s(t) cos(theta) + H{s}(t) sin(theta),  theta = 2 pi nu0 tau_true(t),
    with t found from t + tau_true(t) = t_st by fixed-point iteration;
  * each station adds independent receiver noise: sqrt(rho) x + sqrt(1-rho) n,
    then quantises to 2 bits and packs into frames.

s and H{s} are evaluated off-grid with a 64-tap Kaiser-windowed sinc
interpolator (beta = 8) in float64.  Heavy array work uses torch on the CPU
for its threads; nothing here depends on a GPU.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np
import torch

from . import format as fmt
from .job import Job, Station

TAPS = 64
KAISER_BETA = 8.0


def _polyval(c: Sequence[float], t: np.ndarray) -> np.ndarray:
    """sum_k c[k] t^k (ascending coefficients) in float64."""
    out = np.zeros_like(t, dtype=np.float64)
    for ck in reversed(list(c)):
        out = out * t + ck
    return out


def _splitmix(*vals: int) -> int:
    x = 0x9E3779B97F4A7C15
    for v in vals:
        x = (x ^ (int(v) & 0xFFFFFFFFFFFFFFFF)) & 0xFFFFFFFFFFFFFFFF
        x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
        x = z ^ (z >> 31)
    return x


def seed_of(*vals: int) -> int:
    """Deterministic 63-bit seed from a tuple of integers (SplitMix64 mixing)."""
    return _splitmix(*vals) & 0x7FFFFFFFFFFFFFFF


def buffer_extent(poly: Sequence[float], sub_start: int, n_frames: int, N: int,
                  fs: float, C: int, margin: int) -> tuple[int, int]:
    """(first_sample, n_frames_m5b) covering every window the correlator reads."""
    t = (sub_start + np.linspace(0.0, n_frames * N, 65)) / fs
    D = _polyval(poly, t) * fs
    lo = sub_start + int(math.floor(D.min())) - margin
    hi = sub_start + n_frames * N + int(math.ceil(D.max())) + margin
    spf = fmt.samples_per_frame(C)
    n_m5b = -(-(hi - lo) // spf)
    return lo, n_m5b


_TABLE_PHASES = 4096


def _kernel_table(device="cpu") -> torch.Tensor:
    """Windowed-sinc taps for fractional offsets 0, 1/P, .., 1 (P = 4096), float64 [P+1, 64]."""
    half = TAPS // 2
    fr = torch.arange(_TABLE_PHASES + 1, dtype=torch.float64, device=device) / _TABLE_PHASES
    m = torch.arange(-half + 1, half + 1, dtype=torch.float64, device=device)   # -31 .. 32
    x = fr[:, None] - m[None, :]
    win = torch.special.i0(KAISER_BETA * torch.sqrt(torch.clamp(1.0 - (x / half) ** 2, min=0.0)))
    return torch.sinc(x) * win / float(np.i0(KAISER_BETA))


def _interp(sig: torch.Tensor, u: torch.Tensor, chunk: int = 1 << 18) -> torch.Tensor:
    """Windowed-sinc interpolation of sig (float64 or complex128, grid 0..len-1) at
    fractional indices u.

    Taps come from a 4096-phase table, linearly interpolated between phases
    (tap error below 1e-8 of the peak tap).
    """
    half = TAPS // 2
    table = _kernel_table(sig.device)
    rows = sig.unfold(0, TAPS, 1)                                        # rows[i] = sig[i .. i+63]
    out = torch.empty(u.shape[0], dtype=sig.dtype, device=sig.device)
    for a in range(0, u.shape[0], chunk):
        uu = u[a:a + chunk]
        idx = torch.floor(uu)
        p = (uu - idx) * _TABLE_PHASES
        pi = torch.clamp(torch.floor(p), max=_TABLE_PHASES - 1)
        w = (p - pi)[:, None]
        pi = pi.to(torch.int64)
        h = (table[pi] * (1.0 - w) + table[pi + 1] * w).to(sig.dtype)
        win = rows[idx.to(torch.int64) - half + 1]
        out[a:a + chunk] = (win * h).sum(dim=1)
    return out


def two_station_job(*, fs: float, N: int, n_frames: int, sub_start: int,
                    model_polys: List[Sequence[float]], residual_delay_s: List[float],
                    lo_hz: float, rho: float, seed: int, C: int = 1,
                    margin: int = 1024, poly_span=(0.0, 120.0), name: str = "",
                    device="cpu") -> Job:
    """Single-subband, single-pol job with a common sky signal (exact physics).

    Works for any number of stations (the name reflects the usual use).  The
    torch parts (sky FFT, interpolation, noise, packing) run on `device`; the
    recordings are returned on that device.
    """
    n_st = len(model_polys)
    assert C == 1, "exact-physics generator records one stream"
    extents = [buffer_extent(p, sub_start, n_frames, N, fs, C, margin) for p in model_polys]
    spf = fmt.samples_per_frame(C)

    # reference times of every station sample (fixed point of t + tau_true(t) = t_st)
    t_ref = []
    for (first, n_m5b), poly, dlt in zip(extents, model_polys, residual_delay_s):
        j = first + np.arange(n_m5b * spf, dtype=np.int64)
        t_st = j.astype(np.float64) / fs
        t = t_st - (_polyval(poly, t_st) + dlt)
        for _ in range(4):
            t = t_st - (_polyval(poly, t) + dlt)
        t_ref.append(t)

    # sky on the reference grid, covering all stations' reference times
    k_lo = int(math.floor(min(t.min() for t in t_ref) * fs)) - TAPS
    k_hi = int(math.ceil(max(t.max() for t in t_ref) * fs)) + TAPS
    n_sky = k_hi - k_lo
    g = torch.Generator().manual_seed(seed_of(seed, 0x5C7))
    s = torch.randn(n_sky, generator=g, dtype=torch.float64).to(device)
    spec = torch.fft.fft(s)
    h = torch.zeros(n_sky, dtype=torch.float64, device=device)
    h[0] = 1.0
    if n_sky % 2 == 0:
        h[n_sky // 2] = 1.0
        h[1:n_sky // 2] = 2.0
    else:
        h[1:(n_sky + 1) // 2] = 2.0
    analytic = torch.fft.ifft(spec * h)                                  # s + i H{s}

    stations = []
    for si, ((first, n_m5b), poly, dlt, t) in enumerate(zip(extents, model_polys,
                                                             residual_delay_s, t_ref)):
        u = torch.from_numpy(t * fs - k_lo).to(device)
        z = _interp(analytic, u)
        s_i, h_i = z.real, z.imag
        # theta = 2 pi frac(nu0 * tau_true(t)); long double keeps the fraction exact enough
        tau = _polyval(poly, t) + dlt
        ph = np.longdouble(lo_hz) * tau.astype(np.longdouble)
        ph = (ph - np.floor(ph)).astype(np.float64)
        th = torch.from_numpy(2.0 * np.pi * ph).to(device)
        x = s_i * torch.cos(th) + h_i * torch.sin(th)
        gn = torch.Generator().manual_seed(seed_of(seed, 0x401, si))
        noise = torch.randn(x.shape[0], generator=gn, dtype=torch.float64).to(device)
        v = math.sqrt(rho) * x + math.sqrt(1.0 - rho) * noise
        codes = fmt.quantise(v)[None, :]
        frames = fmt.frame_codes(codes, C, first, fs, si)
        stations.append(Station(frames=frames, first_sample=first,
                                delay_poly=np.asarray(poly, dtype=np.float64),
                                poly_span=poly_span, station_id=si))
    return Job(n_stations=n_st, n_subbands=1, n_pols=1, n_chan=N // 2, n_streams=C,
               stream_map=[0], fs_hz=fs, lo_hz=[lo_hz], sub_start=sub_start,
               n_frames=n_frames, stations=stations, name=name)
