"""GPU parity: delay-rate fringe search (xc_fringe_search) against oracle/fringe.py.

Maps are compared element by element; peaks by validity (the GPU's bin must be a
maximum of the oracle's map to FP32 rounding; equal to the oracle's bin when that
maximum is clear) and by amplitude, phase and refined position.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import fringe, fx
from synth import configs

pytestmark = pytest.mark.gpu


def _tone(T, n_chan, D, R, d0, r0, amp=1.0, phase=0.0):
    t = np.arange(T)[:, None]
    k = np.arange(n_chan)[None, :]
    return amp * np.exp(2j * np.pi * (k * d0 / D + t * r0 / R) + 1j * phase)


def _vis_set(rng, T, n_sb, nbl, n_chan, D, R, noise=0.3):
    V = noise * (rng.normal(size=(T, n_sb, nbl, n_chan)) + 1j * rng.normal(size=(T, n_sb, nbl, n_chan)))
    truth = {}
    for sb in range(n_sb):
        for bl in range(nbl):
            d0 = int(rng.integers(-D // 2 + 2, D // 2 - 2))
            r0 = int(rng.integers(-R // 2 + 1, R // 2 - 1)) if R >= 4 else 0
            V[:, sb, bl, :] += _tone(T, n_chan, D, R, d0 + rng.uniform(-0.4, 0.4),
                                     r0 + rng.uniform(-0.4, 0.4), amp=1.0 + 0.1 * bl,
                                     phase=rng.uniform(-3, 3))
            truth[sb, bl] = (d0, r0)
    return V


def _check(corr, V, D, R, dnu, tint, dw=0, rw=0, map_tol=2e-5):
    peaks_o, G = fringe.fringe_search(V, D, R, dnu, tint, dw, rw)
    vis = torch.from_numpy(V.astype(np.complex64)).cuda()
    peaks, gmap = corr.fringe_search(vis, D, R, dnu, tint, dw, rw, want_map=True)
    Gg = gmap.cpu().numpy()
    scale = np.abs(G).max()
    assert np.max(np.abs(Gg - G)) <= map_tol * scale
    n_sb, nbl = peaks.shape
    for sb in range(n_sb):
        for bl in range(nbl):
            p, po = peaks[sb, bl], peaks_o[sb][bl]
            A = np.abs(G[sb, bl])
            d, r = int(p["delay_bin"]) % D, int(p["rate_bin"]) % R
            mask = fringe._window_mask(R, D, dw, rw)
            assert mask[r, d]
            amax = A[mask].max()
            assert A[r, d] >= amax * (1 - 1e-5)               # a valid maximum
            second = np.sort(A[mask].ravel())[-2]
            if amax > second * (1 + 1e-4):                    # a clear maximum: the same bin
                assert (p["delay_bin"], p["rate_bin"]) == (po.delay_bin, po.rate_bin)
                assert abs(p["amp"] - po.amp) <= 1e-5 * po.amp + 1e-7
                if po.amp > 1e-3:
                    assert abs(np.angle(np.exp(1j * (p["phase"] - po.phase)))) < 1e-3
                    assert abs(p["delay_off"] - po.delay_off) < 2e-3
                    assert abs(p["rate_off"] - po.rate_off) < 2e-3
                    assert abs(p["delay_s"] - po.delay_s) <= 2e-3 / (D * dnu)
                    assert abs(p["rate_hz"] - po.rate_hz) <= 2e-3 / (R * tint)
    return peaks, peaks_o


@pytest.fixture(scope="module")
def xc():
    from paper_1502_06894_amd import xcorr
    return xcorr


@pytest.fixture(scope="module")
def corr(xc):
    return xc.Correlator(0)


@pytest.mark.parametrize("T,n_sb,nbl,n_chan,D,R", [
    (12, 2, 3, 200, 512, 32),        # ragged channel count, both axes padded
    (5, 1, 4, 256, 256, 8),          # no delay padding
    (1, 1, 2, 128, 1024, 1),         # a single sub-integration
    (64, 1, 2, 1024, 2048, 64),      # the C2 channel count, no rate padding
    (100, 1, 2, 300, 4096, 128),     # rate FFT of a ragged sub-integration count
    (256, 1, 1, 512, 512, 1024),     # the largest rate transform, 256 sub-integrations
    (3, 2, 2, 1000, 16384, 4),       # the largest delay transform; a four-point rate axis
    (2, 1, 3, 64, 8192, 2),          # two sub-integrations
])
def test_fringe_parity(corr, T, n_sb, nbl, n_chan, D, R):
    rng = np.random.default_rng(T * 1000 + D)
    V = _vis_set(rng, T, n_sb, nbl, n_chan, D, R)
    _check(corr, V, D, R, 15625.0, 0.5)


def test_fringe_window(corr):
    T, n_chan, D, R = 8, 128, 512, 16
    V = np.zeros((T, 1, 2, n_chan), complex)
    V[:, 0, 0] = _tone(T, n_chan, D, R, 200, 6) + _tone(T, n_chan, D, R, -20, -2, amp=0.4)
    V[:, 0, 1] = _tone(T, n_chan, D, R, -230, -7, amp=0.8) + _tone(T, n_chan, D, R, 3, 1, amp=0.3)
    peaks, _ = _check(corr, V, D, R, 1.0, 1.0, dw=32, rw=3)
    assert (peaks[0, 0]["delay_bin"], peaks[0, 0]["rate_bin"]) == (-20, -2)
    assert (peaks[0, 1]["delay_bin"], peaks[0, 1]["rate_bin"]) == (3, 1)


def test_fringe_errors(corr, xc):
    vis = torch.zeros((4, 1, 1, 128), dtype=torch.complex64, device="cuda")
    for kw in [dict(delay_len=100), dict(delay_len=64), dict(rate_len=2), dict(rate_len=4096)]:
        a = dict(delay_len=256, rate_len=8)
        a.update(kw)
        with pytest.raises(xc.XcError) as e:
            corr.fringe_search(vis, a["delay_len"], a["rate_len"], 1.0, 1.0)
        assert e.value.code == xc.XC_E_INVAL
    with pytest.raises(xc.XcError) as e:
        corr.fringe_search(vis, 256, 8, 1.0, 1.0,
                           workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert e.value.code == xc.XC_E_NOMEM


def test_fringe_on_gpu_correlated_physics(xc, corr):
    """Eight 750-frame sub-integrations of the exact-physics C1 generator correlated
    on the GPU, then searched on the GPU: the space baseline's fringe at the injected
    residual delay, and the search equal to the oracle's search of the same input."""
    job = configs.c1_job(n_frames=6000, device="cuda")
    xc.job_to_device(job)
    N, fs, sub = job.N, job.fs_hz, 750
    vs = []
    for a in range(0, job.n_frames, sub):
        part = dataclasses.replace(job, sub_start=job.sub_start + a * N, n_frames=sub)
        vis, w = corr.correlate(part)
        vs.append(vis)
    V = torch.stack(vs)                                   # [T, 1, 3, n_chan]
    D, R = 4 * job.n_chan, 16
    dnu, tint = fs / N, sub * N / fs
    peaks, peaks_o = _check(corr, V.cpu().numpy().astype(np.complex128), D, R, dnu, tint)
    bl = fx.baseline_index(0, 1, 2)
    p = peaks[0, bl]
    t_mid = (job.sub_start + job.n_frames * N / 2) / fs
    rate = sum(k * c * t_mid ** (k - 1) for k, c in enumerate(configs.SPACE_C1) if k > 0)
    lag = configs.C1_RESIDUAL_SAMPLES / (1.0 + rate)
    assert abs(p["delay_s"] * fs - lag) < 0.15
