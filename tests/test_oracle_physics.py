"""Oracle pin: end-to-end physics on the exact-physics two-station generator.

The space station's true delay exceeds its model by delta = 137.25 samples
(defined in reference time).  A residual delay defined in reference time
appears in the sky signal as a lag of delta / (1 + tau'), tau' being the
space station's delay rate, so the lag spectrum of V_01 must peak at
m = delta fs / (1 + tau') samples with phase 2 pi frac(nu0 delta / (1 + tau')).
The fringe amplitude is the analog correlation coefficient 0.05 times the
4-level quantiser's efficiency (0.8825 for thresholds +-0.9816 sigma and outer
level 3.3359) times the FX frame overlap 1 - lag/N.
"""
import numpy as np
import pytest

from oracle import fx
from synth import configs


def _lag_spectrum(v, N, m):
    k = np.arange(v.shape[0])
    return np.exp(-2j * np.pi * np.outer(m, k) / N) @ v


@pytest.fixture(scope="module")
def c1_small():
    job = configs.c1_job(n_frames=6000)
    V, W = fx.correlate(job)
    return job, V, W


def test_fringe_peak_delay_and_phase(c1_small):
    job, V, W = c1_small
    N, fs = job.N, job.fs_hz
    v = V[0, fx.baseline_index(0, 1, 2)]
    m = np.arange(0, N, 1.0 / 16)                       # zero-padded x16 lag grid
    L = _lag_spectrum(v, N, m)
    i = int(np.argmax(np.abs(L)))
    t_mid = (job.sub_start + job.n_frames * N / 2) / fs
    rate = sum(k * c * t_mid ** (k - 1) for k, c in enumerate(configs.SPACE_C1) if k > 0)
    lag = configs.C1_RESIDUAL_SAMPLES / (1.0 + rate)
    assert abs(m[i] - lag) <= 0.05
    assert abs(m[i] - configs.C1_RESIDUAL_SAMPLES) <= 0.05
    # phase at the exact lag
    Lx = _lag_spectrum(v, N, np.array([lag]))[0]
    want = (job.lo_hz[0] * lag / fs) % 1.0
    got = (np.angle(Lx) / (2 * np.pi)) % 1.0
    err = (got - want + 0.5) % 1.0 - 0.5
    a0, a1 = V[0, 0].real, V[0, 2].real
    rho = np.abs(Lx) / np.sum(np.sqrt(a0 * a1))
    n_samp = W[0, 1] * N
    sigma = 1.0 / (rho * np.sqrt(n_samp))               # phase noise (rad) of the band sum
    assert abs(err) * 2 * np.pi < max(4 * sigma, 0.02)
    # detected coefficient: 0.05 x 0.8825, times the frame overlap 1 - lag/N of an FX
    # correlator (the lagged station shares only N - lag samples of each frame), less a
    # few per cent of interpolation and image-leakage losses
    expect = 0.05 * 0.8825 * (1.0 - lag / N)
    assert 0.85 * expect < rho < 1.05 * expect


def test_white_noise_autos_flat_c1(c1_small):
    job, V, W = c1_small
    E = job.N * 4.30481
    for bl in (0, 2):
        A = V[0, bl].real[8:]                           # leave out channels near DC
        assert abs(A.mean() / E - 1) < 5e-3
        assert A.std() / E < 2.0 / np.sqrt(W[0, bl])


def test_opposite_residual_flips_peak():
    job = configs.c1_job(n_frames=600, seed=99)
    job.stations = job.stations[::-1]                    # space first: the lag changes sign
    V, _ = fx.correlate(job)
    N = job.N
    m = np.arange(-N // 2, N // 2, 0.25)
    L = _lag_spectrum(V[0, 1], N, m)
    assert abs(m[np.argmax(np.abs(L))] + 137.25) <= 0.25
