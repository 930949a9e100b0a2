"""Oracle pins: delay-rate fringe search (oracle/fringe.py, steps F1-F7).

Pinned by closed forms (a fringe of known delay, rate, amplitude and phase of
either sign), a brute-force two-dimensional DFT, the window and tie rules, the
sub-bin refinement on off-grid fringes, and end to end by the exact-physics
two-station generator: stacked sub-integrations of the space baseline must put
the fringe at the injected residual delay.
"""
import numpy as np
import pytest

from oracle import fringe, fx
from synth import configs


def _tone(T, n_sb, nbl, n_chan, D, R, d0, r0, amp=1.0, phase=0.0):
    t = np.arange(T)[:, None, None, None]
    k = np.arange(n_chan)[None, None, None, :]
    v = amp * np.exp(2j * np.pi * (k * d0 / D + t * r0 / R) + 1j * phase)
    return np.broadcast_to(v, (T, n_sb, nbl, n_chan)).copy()


@pytest.mark.parametrize("d0,r0", [(37, 5), (-101, -3), (0, 0), (-1, 7)])
def test_tone_closed_form(d0, r0):
    T, n_chan, D, R = 12, 128, 512, 32
    dnu, tint = 15625.0, 0.25
    V = _tone(T, 1, 2, n_chan, D, R, d0, r0, amp=0.37, phase=1.1)
    peaks, G = fringe.fringe_search(V, D, R, dnu, tint)
    for p in peaks[0]:
        assert (p.delay_bin, p.rate_bin) == (d0, r0)
        assert abs(p.amp - 0.37) < 1e-12
        assert abs(np.angle(np.exp(1j * (p.phase - 1.1)))) < 1e-12
        # on-grid fringe: the neighbours of the peak are equal, no sub-bin offset
        assert abs(p.delay_off) < 1e-9 and abs(p.rate_off) < 1e-9
        assert abs(p.delay_s - d0 / (D * dnu)) < 1e-9 / (D * dnu)
        assert abs(p.rate_hz - r0 / (R * tint)) < 1e-9


def test_map_matches_brute_force_dft():
    rng = np.random.default_rng(11)
    T, n_sb, nbl, n_chan, D, R = 3, 2, 3, 8, 16, 4
    V = rng.normal(size=(T, n_sb, nbl, n_chan)) + 1j * rng.normal(size=(T, n_sb, nbl, n_chan))
    G = fringe.delay_rate_map(V, D, R)
    Gb = np.zeros((n_sb, nbl, R, D), complex)
    for sb in range(n_sb):
        for bl in range(nbl):
            for r in range(R):
                for d in range(D):
                    s = 0j
                    for t in range(T):
                        for k in range(n_chan):
                            s += V[t, sb, bl, k] * np.exp(-2j * np.pi * (k * d / D + t * r / R))
                    Gb[sb, bl, r, d] = s
    assert np.max(np.abs(G - Gb)) < 1e-10 * np.max(np.abs(Gb))


def test_window_and_tie_rule():
    T, n_chan, D, R = 8, 128, 256, 16
    a = _tone(T, 1, 1, n_chan, D, R, 90, 6, amp=1.0)
    b = _tone(T, 1, 1, n_chan, D, R, 10, -2, amp=0.5)
    peaks, _ = fringe.fringe_search(a + b, D, R, 1.0, 1.0)
    assert (peaks[0][0].delay_bin, peaks[0][0].rate_bin) == (90, 6)
    peaks, _ = fringe.fringe_search(a + b, D, R, 1.0, 1.0, delay_win=40, rate_win=4)
    assert (peaks[0][0].delay_bin, peaks[0][0].rate_bin) == (10, -2)
    # an all-zero map ties everywhere: the first row-major index wins, and inside a
    # window that excludes bin (0, 0) the first index of the window
    z = np.zeros((T, 1, 1, n_chan), complex)
    peaks, _ = fringe.fringe_search(z, D, R, 1.0, 1.0)
    assert (peaks[0][0].delay_bin, peaks[0][0].rate_bin, peaks[0][0].amp) == (0, 0, 0.0)
    m = fringe._window_mask(R, D, 3, 2)
    r, d = divmod(int(np.argmax(m)), D)
    assert (fringe.signed(d, D), fringe.signed(r, R)) == (0, 0)


@pytest.mark.parametrize("frac", [0.2, 0.35, -0.3])
def test_refinement_moves_toward_an_off_grid_fringe(frac):
    T, n_chan, D, R = 16, 256, 1024, 64
    d_true, r_true = 77 + frac, -9 - frac
    V = _tone(T, 1, 1, n_chan, D, R, d_true, r_true)
    p = fringe.fringe_search(V, D, R, 1.0, 1.0)[0][0][0]
    assert abs(p.delay_bin + p.delay_off - d_true) < abs(p.delay_bin - d_true)
    assert abs(p.rate_bin + p.rate_off - r_true) < abs(p.rate_bin - r_true)


def test_physics_fringe_at_injected_delay():
    """Eight 750-frame sub-integrations of the exact-physics C1 generator: the
    space baseline's fringe sits at delta / (1 + tau') samples."""
    job = configs.c1_job(n_frames=6000)
    N, fs = job.N, job.fs_hz
    sub = 750
    Vs = []
    for a in range(0, job.n_frames, sub):
        V, W = fx.correlate(job, frames=np.arange(a, a + sub), threads=8)
        Vs.append(V)
    V = np.stack(Vs)                                    # [T, sb, bl, k]
    D, R = 4 * job.n_chan, 16
    dnu, tint = fs / N, sub * N / fs
    peaks, G = fringe.fringe_search(V, D, R, dnu, tint)
    bl = fx.baseline_index(0, 1, 2)
    p = peaks[0][bl]
    t_mid = (job.sub_start + job.n_frames * N / 2) / fs
    rate = sum(k * c * t_mid ** (k - 1) for k, c in enumerate(configs.SPACE_C1) if k > 0)
    lag = configs.C1_RESIDUAL_SAMPLES / (1.0 + rate)
    assert abs(p.delay_s * fs - lag) < 0.15             # bins are 0.5 samples wide
    assert abs(p.rate_hz) < 1.0 / (R * tint)            # a constant residual: no rate
    # a single peak, well above the rest of the map
    A = np.abs(G[0, bl])
    assert A.max() > 8.0 * np.median(A)
