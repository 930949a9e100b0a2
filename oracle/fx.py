"""FX correlation, steps O1-O11, in float64 (long double for the fringe phase).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Citations refer to the paper's sections: the abstract (FX architecture:
Fourier transform first, then cross-multiply), section 2's data-format
paragraph (recordings converted to Mark5B so the correlator can read them) and
its delay-model paragraphs (delays for an antenna with arbitrary, changing
position and velocity, relativistic terms, and the spacecraft-to-tracking
station transmission delay, all of which arrive here summed into one delay
polynomial per station).  The paper gives no formulas; each step states the
convention it fixes.  O11 (optional per station) is the correction of the
spacecraft's acceleration-era delay drift that the paper lists among its
future improvements (section 2, the closing list).
"""
from __future__ import annotations

import os
from typing import Iterable, Optional, Sequence

import numpy as np
import scipy.fft

SYNC_WORD = 0xABADDEED
HEADER_WORDS = 4
PAYLOAD_WORDS = 2500
# 2-bit levels, offset binary; the +-3.3359 magnitude is the single-precision
# constant widened to double so that both correlator paths use one value.
LEVELS = np.array([-3.3359, -1.0, 1.0, 3.3359], dtype=np.float32).astype(np.float64)

_WORKERS = os.cpu_count() or 1


# ----------------------------------------------------------------- recording format

def as_words(frames) -> np.ndarray:
    """Frames (torch or numpy, int32 or uint32, [n_m5b, 2504]) as numpy uint32."""
    if hasattr(frames, "detach"):
        frames = frames.detach().cpu().numpy()
    return np.ascontiguousarray(frames).view(np.uint32)


def samples_per_frame(C: int) -> int:
    return PAYLOAD_WORDS * 16 // C


def unpack_codes(words: np.ndarray, C: int, stream: int, pos: np.ndarray) -> np.ndarray:
    """O5 (format): 2-bit code of `stream` at per-stream sample positions `pos`.

    Payload word w (counted over the whole recording, headers excluded) holds
    16 fields; field j is stream j mod C at sample w*(16/C) + j div C.
    """
    spf = samples_per_frame(C)
    spw = 16 // C
    pos = np.asarray(pos, dtype=np.int64)
    fm = pos // spf
    ip = pos - fm * spf
    w = ip // spw
    sub = ip - w * spw
    field = sub * C + stream
    word = words[fm, HEADER_WORDS + w]
    return ((word >> (2 * field).astype(np.uint32)) & np.uint32(3)).astype(np.uint8)


def sync_ok(words: np.ndarray) -> np.ndarray:
    """A0: per-frame validity from the sync word."""
    return words[:, 0] == np.uint32(SYNC_WORD)


# ----------------------------------------------------------------- delay model

def horner(coeffs: Sequence[float], t: np.ndarray) -> np.ndarray:
    """O2: r = c_d; r = r*t + c_k for k = d-1 .. 0, one rounding per operation."""
    c = [np.float64(x) for x in coeffs]
    r = np.full(np.shape(t), c[-1], dtype=np.float64)
    for ck in reversed(c[:-1]):
        r = r * t          # rounded product
        r = r + ck         # rounded sum (numpy never fuses the two)
    return r


def frame_delays(delay_poly, sub_start: int, N: int, fs: float,
                 frames: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """O1-O3 for the given frame indices: (n_int int64, d float64).

    t_mid is the reference time of the frame's centre sample; tau(t) is the
    delay at which the wavefront reaches the station; D = tau*fs samples;
    n_int rounds half up; d = D - n_int lies in [-1/2, 1/2) and is exact.
    """
    f = np.asarray(frames, dtype=np.int64)
    num = np.int64(sub_start) + f * np.int64(N) + np.int64(N // 2)     # exact integer
    t_mid = num.astype(np.float64) / np.float64(fs)                      # one division
    tau = horner(delay_poly, t_mid)
    D = tau * np.float64(fs)
    n_int = np.floor(D + np.float64(0.5)).astype(np.int64)
    d = D - n_int.astype(np.float64)
    return n_int, d


def frame_valid(words: np.ndarray, C: int, first_sample: int, sub_start: int, N: int,
                frames: np.ndarray, n_int: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """O4: (base, valid).  base is the window start inside the recording; the
    frame is valid iff the whole window lies inside the recording and every
    recording frame it touches has a good sync word (validity is per whole FFT
    frame; a partly bad window is dropped)."""
    spf = samples_per_frame(C)
    n_samples = words.shape[0] * spf
    f = np.asarray(frames, dtype=np.int64)
    base = np.int64(sub_start) + f * np.int64(N) + n_int - np.int64(first_sample)
    valid = (base >= 0) & (base + N <= n_samples)
    good = sync_ok(words)
    for i in np.nonzero(valid)[0]:
        a, b = base[i] // spf, (base[i] + N - 1) // spf
        if not good[a:b + 1].all():
            valid[i] = False
    return base, valid


def frame_rates(delay_poly, sub_start: int, N: int, fs: float, frames: np.ndarray) -> np.ndarray:
    """O11 input: the delay rate rho = tau'(t_mid) (s/s, i.e. samples of delay per
    sample) at each frame's centre, from the derivative polynomial by Horner."""
    f = np.asarray(frames, dtype=np.int64)
    num = np.int64(sub_start) + f * np.int64(N) + np.int64(N // 2)
    t_mid = num.astype(np.float64) / np.float64(fs)
    c = np.asarray(delay_poly, dtype=np.float64)
    if c.shape[0] < 2:
        return np.zeros(f.shape[0])
    dc = c[1:] * np.arange(1, c.shape[0], dtype=np.float64)
    return horner(dc, t_mid)


def rate_corrected(X: np.ndarray, Xr: np.ndarray, rho: np.ndarray, k: np.ndarray, N: int):
    """O11: first-order correction of the delay's drift inside a frame.

    Inside frame f the delay is D_c + rho (n - N/2) samples, while the window
    and the fractional-delay phase take D_c for the whole frame.  The aligned
    samples are therefore the window resampled about the frame centre,
    a(n) = w(N/2 + (1 + rho)(n - N/2) + d), whose spectrum to first order in rho
    is (1 - rho) W(k) + (2 pi i rho k / N) Wr(k), with Wr the spectrum of
    (n - N/2) w(n).  X, Xr: [nf, K] spectra of w and of the ramp-weighted
    window; rho: [nf]; k: [K] (signed for a full band).
    """
    r = np.asarray(rho, dtype=np.float64)[:, None]
    return (1.0 - r) * X + (2j * np.pi / N) * r * np.asarray(k, dtype=np.float64)[None, :] * Xr


# ----------------------------------------------------------------- per-sample fringe phase

def _horner_ld(coeffs, t: np.ndarray) -> np.ndarray:
    c = [np.longdouble(x) for x in coeffs]
    r = np.full(t.shape, c[-1], dtype=np.longdouble)
    for ck in reversed(c[:-1]):
        r = r * t + ck
    return r


def fringe_phase(delay_poly, phase_poly_sb, lo_hz: float, sub_start: int, N: int,
                 fs: float, frames: np.ndarray) -> np.ndarray:
    """O6 phase, in turns wrapped to [0, 1), for every sample of each frame.

    t_n = (j0 + f N + n) / fs is the reference time of sample n; the phase is
    nu_sb * tau(t_n) (or the explicit phase polynomial at t_n), evaluated in
    x86 long double so that the fraction of a ~1e9-turn phase stays exact to
    ~1e-10 turns.
    """
    f = np.asarray(frames, dtype=np.int64)
    num = np.int64(sub_start) + f[:, None] * np.int64(N) + np.arange(N, dtype=np.int64)[None, :]
    t = num.astype(np.longdouble) / np.longdouble(fs)
    if phase_poly_sb is not None:
        phi = _horner_ld(phase_poly_sb, t)
    else:
        phi = np.longdouble(lo_hz) * _horner_ld(delay_poly, t)
    return (phi - np.floor(phi)).astype(np.float64)


# ----------------------------------------------------------------- per-station spectra

def rotated_samples(job, s: int, sb: int, p: int, frames: np.ndarray, *,
                    rotate: bool = True, words: Optional[np.ndarray] = None):
    """O1-O6 for station s, input (sb, p): (y [nf, N] complex128, d [nf], valid [nf]).

    Rows of invalid frames are zero.
    """
    st = job.stations[s]
    N, C, fs = job.N, job.n_streams, job.fs_hz
    if words is None:
        words = as_words(st.frames)
    f = np.asarray(frames, dtype=np.int64)
    n_int, d = frame_delays(st.delay_poly, job.sub_start, N, fs, f)          # O1-O3
    base, valid = frame_valid(words, C, st.first_sample, job.sub_start, N, f, n_int)   # O4
    y = np.zeros((f.shape[0], N), dtype=np.complex128)
    vi = np.nonzero(valid)[0]
    if vi.size == 0:
        return y, d, valid
    stream = job.stream_map[sb * job.n_pols + p]
    pos = base[vi, None] + np.arange(N, dtype=np.int64)[None, :]
    q = LEVELS[unpack_codes(words, C, stream, pos)]                        # O5
    if rotate:                                                             # O6
        pp = None if st.phase_poly is None else st.phase_poly[sb]
        ph = fringe_phase(st.delay_poly, pp, job.lo_hz[sb], job.sub_start, N, fs, f[vi])
        y[vi] = q * np.exp(2j * np.pi * ph)
    else:
        y[vi] = q
    return y, d, valid


def station_spectra(job, s: int, sb: int, p: int, frames: np.ndarray, *,
                    rotate: bool = True, frac: bool = True,
                    full_band: bool = False, words: Optional[np.ndarray] = None):
    """O1-O8 for station s, input (sb, p): (Y [nf, K] complex128, valid [nf]).

    K = N/2 channels (DC up to, not including, Nyquist), or all N bins with
    full_band (then the fractional-delay phase uses signed frequencies).
    Invalid frames give zero spectra.
    """
    N = job.N
    y, d, valid = rotated_samples(job, s, sb, p, frames, rotate=rotate, words=words)
    K = N if full_band else N // 2
    Y = scipy.fft.fft(y, axis=1, workers=_WORKERS)[:, :K]                   # O7
    k = np.arange(K, dtype=np.float64)
    if full_band:
        k = np.where(k < N // 2, k, k - N)
    st = job.stations[s]
    if getattr(st, "rate_correct", False):                                 # O11
        ramp = np.arange(N, dtype=np.float64) - N // 2
        Yr = scipy.fft.fft(y * ramp[None, :], axis=1, workers=_WORKERS)[:, :K]
        rho = frame_rates(st.delay_poly, job.sub_start, N, job.fs_hz, frames)
        Y = rate_corrected(Y, Yr, rho, k, N)
    if frac:                                                               # O8
        Y = Y * np.exp(2j * np.pi * k[None, :] * d[:, None] / N)
    Y[~valid] = 0.0
    return Y, valid


# ----------------------------------------------------------------- correlate

def baseline_index(i: int, j: int, M: int) -> int:
    return i * M - i * (i - 1) // 2 + (j - i)



def _partial_sums(job, sb, ins, fc, words, rotate, frac, full_band):
    """O9 over one chunk of frames: (sum of Y_a conj(Y_b) [m, m, K], pair counts [m, m])."""
    P = job.n_pols
    Ys, vs = [], []
    for i in ins:
        Y, v = station_spectra(job, i // P, sb, i % P, fc, rotate=rotate, frac=frac,
                               full_band=full_band, words=words[i // P])
        Ys.append(Y)
        vs.append(v)
    Ya = np.stack(Ys)                                              # [m, nf, K]
    va = np.stack(vs).astype(np.int64)                             # [m, nf]
    return np.einsum("afk,bfk->abk", Ya, np.conj(Ya)), va @ va.T


def correlate(job, *, subbands: Optional[Iterable[int]] = None,
              inputs: Optional[Iterable[int]] = None,
              frames: Optional[np.ndarray] = None, chunk: int = 256,
              rotate: bool = True, frac: bool = True, full_band: bool = False,
              threads: int = 1):
    """O9-O10: (V complex128 [n_sb, M(M+1)/2, K], W int64 [n_sb, M(M+1)/2]).

    Inputs are ordered i = s*P + p.  V_ij is the mean over frames valid for
    both stations of Y_i conj(Y_j) (unnormalised FFT); W_ij counts those
    frames; W = 0 gives V = 0.  Entries not requested (subbands/inputs
    subsets) are NaN in V and -1 in W.  `frames` defaults to 0..n_frames-1.
    `threads` > 1 evaluates frame chunks concurrently; partial sums are still
    added in chunk order.
    """
    M = job.M
    P = job.n_pols
    K = job.N if full_band else job.n_chan
    nbl = M * (M + 1) // 2
    sbs = list(range(job.n_subbands)) if subbands is None else list(subbands)
    ins = list(range(M)) if inputs is None else sorted(set(inputs))
    fr = np.arange(job.n_frames, dtype=np.int64) if frames is None else np.asarray(frames, np.int64)
    V = np.full((job.n_subbands, nbl, K), np.nan + 1j * np.nan, dtype=np.complex128)
    W = np.full((job.n_subbands, nbl), -1, dtype=np.int64)
    words = {s: as_words(job.stations[s].frames) for s in sorted({i // P for i in ins})}
    chunks = [fr[a:a + chunk] for a in range(0, fr.shape[0], chunk)]
    for sb in sbs:
        def work(fc, sb=sb):
            return _partial_sums(job, sb, ins, fc, words, rotate, frac, full_band)
        if threads > 1:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(threads) as ex:
                parts = list(ex.map(work, chunks))
        else:
            parts = [work(fc) for fc in chunks]
        Vs = np.zeros((len(ins), len(ins), K), dtype=np.complex128)
        Ws = np.zeros((len(ins), len(ins)), dtype=np.int64)
        for v, w in parts:                                         # fixed chunk order
            Vs += v
            Ws += w
        for ai, i in enumerate(ins):
            for bi, j in enumerate(ins):
                if i > j:
                    continue
                bl = baseline_index(i, j, M)
                W[sb, bl] = Ws[ai, bi]
                V[sb, bl] = Vs[ai, bi] / Ws[ai, bi] if Ws[ai, bi] > 0 else 0.0   # O10
    return V, W
