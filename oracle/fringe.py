"""Delay-rate fringe search over stacked sub-integrations, in float64.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper's first-fringe result is a single peak in the fringe amplitude as a
function of residual delay and residual rate, found inside a fringe-search
window, and its capability list adds wide search windows (section 2, first
fringes; the list of what the space-VLBI correlator can do).  It gives no
formulas; the steps and conventions fixed here:

F1  delay transform: per sub-integration t, subband and baseline, the channel
    spectrum V_t[k] (k = 0 .. n_chan-1, upper-sideband channels of width dnu)
    zero-padded to D points: F_t[d] = sum_k V_t[k] exp(-2 pi i k d / D).
    A visibility with residual delay tau (V[k] ~ exp(+2 pi i k dnu tau)) peaks
    at d = D dnu tau: bin d is a delay of d / (D dnu) seconds.
F2  rate transform: over sub-integrations t = 0 .. T-1 zero-padded to R:
    G[r, d] = sum_t F_t[d] exp(-2 pi i t r / R).  A fringe turning at nu_f Hz
    (F_t ~ exp(+2 pi i nu_f t t_int)) peaks at r = R nu_f t_int: bin r is a
    rate of r / (R t_int) Hz.
F3  signed bins: d in [-D/2, D/2), r in [-R/2, R/2) (bin b >= n/2 is b - n).
F4  window: only |d| <= delay_win and |r| <= rate_win take part (0 = the whole
    axis: a "wide" window).
F5  peak: the largest |G| in the window; ties go to the smallest row-major
    index r * D + d of the unsigned bins.
F6  refinement: a parabola through |G| at the peak and its two neighbours
    along each axis (cyclic) gives the sub-bin offset
    o = (a[-1] - a[+1]) / (2 (a[-1] - 2 a[0] + a[+1])), 0 when the
    denominator is 0.
F7  outputs: amplitude |G_peak| / (n_chan T) (a unit-modulus fringe gives 1),
    phase arg G_peak in radians, delay (d + o_d) / (D dnu) s, rate
    (r + o_r) / (R t_int) Hz.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Peak:
    delay_bin: int        # signed (F3)
    rate_bin: int         # signed (F3)
    amp: float
    phase: float
    delay_off: float      # F6, in bins
    rate_off: float
    delay_s: float
    rate_hz: float


def delay_rate_map(V: np.ndarray, delay_len: int, rate_len: int) -> np.ndarray:
    """F1-F2: G[sb, bl, r, d] from V[t, sb, bl, k] (complex)."""
    V = np.asarray(V, dtype=np.complex128)
    T, n_chan = V.shape[0], V.shape[-1]
    if delay_len < n_chan or rate_len < T:
        raise ValueError("transform shorter than its input")
    F = np.fft.fft(V, n=delay_len, axis=-1)          # F1 (zero-padded)
    G = np.fft.fft(F, n=rate_len, axis=0)            # F2 (zero-padded)
    return np.moveaxis(G, 0, -2)                     # [sb, bl, r, d]


def signed(b: int, n: int) -> int:
    """F3 (a one-point axis has the single bin 0)."""
    return b - n if b >= (n + 1) // 2 else b


def _window_mask(R: int, D: int, delay_win: int, rate_win: int) -> np.ndarray:
    d = np.array([signed(b, D) for b in range(D)])
    r = np.array([signed(b, R) for b in range(R)])
    md = np.abs(d) <= delay_win if delay_win > 0 else np.ones(D, bool)
    mr = np.abs(r) <= rate_win if rate_win > 0 else np.ones(R, bool)
    return mr[:, None] & md[None, :]


def parabola(am: float, a0: float, ap: float) -> float:
    """F6: vertex offset of the parabola through (-1, am), (0, a0), (1, ap)."""
    den = am - 2.0 * a0 + ap
    return 0.0 if den == 0.0 else (am - ap) / (2.0 * den)


def peak_of(G2: np.ndarray, n_chan: int, n_subints: int, chan_width_hz: float, t_int_s: float,
            delay_win: int = 0, rate_win: int = 0) -> Peak:
    """F4-F7 on one map G2[r, d]."""
    R, D = G2.shape
    A = np.abs(G2)
    A = np.where(_window_mask(R, D, delay_win, rate_win), A, -1.0)
    i = int(np.argmax(A))                            # first maximum, row-major (F5)
    r, d = divmod(i, D)
    a0 = abs(G2[r, d])
    od = parabola(abs(G2[r, (d - 1) % D]), a0, abs(G2[r, (d + 1) % D]))
    orr = parabola(abs(G2[(r - 1) % R, d]), a0, abs(G2[(r + 1) % R, d]))
    ds, rs = signed(d, D), signed(r, R)
    return Peak(delay_bin=ds, rate_bin=rs, amp=a0 / (n_chan * n_subints),
                phase=float(np.angle(G2[r, d])), delay_off=od, rate_off=orr,
                delay_s=(ds + od) / (D * chan_width_hz), rate_hz=(rs + orr) / (R * t_int_s))


def fringe_search(V: np.ndarray, delay_len: int, rate_len: int, chan_width_hz: float,
                  t_int_s: float, delay_win: int = 0, rate_win: int = 0):
    """F1-F7 for every subband and baseline of V[t, sb, bl, k]; returns (peaks[sb][bl], G)."""
    V = np.asarray(V)
    T, n_sb, nbl, n_chan = V.shape
    G = delay_rate_map(V, delay_len, rate_len)
    peaks = [[peak_of(G[sb, bl], n_chan, T, chan_width_hz, t_int_s, delay_win, rate_win)
              for bl in range(nbl)] for sb in range(n_sb)]
    return peaks, G
