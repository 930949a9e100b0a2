"""Oracle pins: unpack, fringe rotation, FFT and fractional delay (O5-O8).

Pinned by the O(N^2) DFT on codes assembled by hand, impulse and tone closed
forms, Parseval's theorem and the d = 0 / zero-phase identities.
"""
import numpy as np
import pytest

from oracle import fx, xf
from tests.helpers import job_from_stations, station_from_codes

FS = 32e6
L3 = float(np.float32(3.3359))


def _levels(codes):
    return np.array([-L3, -1.0, 1.0, L3])[codes]


@pytest.mark.parametrize("N,C", [(64, 1), (256, 4), (1024, 16)])
def test_fft_matches_dft_on_known_codes(N, C):
    rng = np.random.default_rng(N)
    nf = 5
    first = 500_000
    codes = rng.integers(0, 4, size=(C, nf * N + 64))
    st = station_from_codes(codes, C, first, [0.0] * 6)
    job = job_from_stations([st], n_chan=N // 2, n_frames=nf, sub_start=first, C=C,
                            stream_map=[C - 1])
    Y, valid = fx.station_spectra(job, 0, 0, 0, np.arange(nf), rotate=False, frac=False,
                                  full_band=True)
    assert valid.all()
    y = _levels(codes[C - 1, :nf * N].reshape(nf, N))
    ref = xf.dft(y)
    assert np.max(np.abs(Y - ref)) < 1e-12 * np.max(np.abs(ref))


def test_impulse_closed_form():
    N, n0, first = 256, 37, 1_000_000
    codes = np.full((1, 4 * N), 2)
    codes[0, N + n0] = 3                      # frame 1: +1 everywhere, 3.3359 at n0
    st = station_from_codes(codes, 1, first, [0.0] * 6)
    job = job_from_stations([st], n_chan=N // 2, n_frames=3, sub_start=first)
    Y, _ = fx.station_spectra(job, 0, 0, 0, np.arange(3), rotate=False, frac=False)
    k = np.arange(N // 2)
    expect = (L3 - 1.0) * np.exp(-2j * np.pi * k * n0 / N)
    expect[0] += N
    assert np.max(np.abs(Y[1] - expect)) < 1e-11
    assert np.max(np.abs(Y[0] - np.where(k == 0, N, 0))) < 1e-11


def test_rotation_tone_lands_in_one_channel_with_known_phase():
    # constant data (+1) rotated by phi(t) = f1 t turns with f1 = k1 fs / N gives
    # y[n] = exp(2 pi i k1 (j0 + f N + n) / N): all power in channel k1, phase fixed by j0 + f N
    N, k1, first = 512, 19, 1_184_000_000
    j0 = first + 7
    codes = np.full((1, 6 * N), 2)
    f1 = k1 * FS / N
    st = station_from_codes(codes, 1, first, [0.0] * 6, phase_poly=[[0.0, f1]])
    job = job_from_stations([st], n_chan=N // 2, n_frames=4, sub_start=j0)
    Y, _ = fx.station_spectra(job, 0, 0, 0, np.arange(4), frac=False)
    for f in range(4):
        expect = np.zeros(N // 2, complex)
        expect[k1] = N * np.exp(2j * np.pi * ((k1 * (j0 + f * N)) % N) / N)
        assert np.max(np.abs(Y[f] - expect)) < 1e-6 * N
    # the opposite sign would have put the tone at N - k1, outside the kept band
    st2 = station_from_codes(codes, 1, first, [0.0] * 6, phase_poly=[[0.0, -f1]])
    job2 = job_from_stations([st2], n_chan=N // 2, n_frames=1, sub_start=j0)
    Y2, _ = fx.station_spectra(job2, 0, 0, 0, np.arange(1), frac=False)
    assert np.max(np.abs(Y2)) < 1e-6 * N


def test_fractional_delay_sign_and_size():
    # delay (m + 0.25) samples: read at +m, then Y[k] *= exp(+2 pi i k 0.25 / N)
    N, k1, m, first = 512, 23, 40, 1_184_000_000
    j0 = first + 100
    codes = np.full((1, 6 * N), 2)
    f1 = k1 * FS / N
    st = station_from_codes(codes, 1, first, [(m + 0.25) / FS], phase_poly=[[0.0, f1]])
    job = job_from_stations([st], n_chan=N // 2, n_frames=2, sub_start=j0)
    Y0, _ = fx.station_spectra(job, 0, 0, 0, np.arange(2), frac=False)
    Y1, _ = fx.station_spectra(job, 0, 0, 0, np.arange(2), frac=True)
    ratio = Y1[:, k1] / Y0[:, k1]
    assert np.allclose(ratio, np.exp(2j * np.pi * k1 * 0.25 / N), atol=1e-9)
    # and with d = 0 (integer delay) the correction is the identity
    st0 = station_from_codes(codes, 1, first, [m / FS], phase_poly=[[0.0, f1]])
    job0 = job_from_stations([st0], n_chan=N // 2, n_frames=2, sub_start=j0)
    A, _ = fx.station_spectra(job0, 0, 0, 0, np.arange(2), frac=False)
    B, _ = fx.station_spectra(job0, 0, 0, 0, np.arange(2), frac=True)
    assert np.max(np.abs(A - B)) < 1e-6


def test_parseval_and_zero_phase_identity():
    rng = np.random.default_rng(3)
    N, first = 1024, 2_000_000
    codes = rng.integers(0, 4, size=(1, 8 * N))
    st = station_from_codes(codes, 1, first, [3.3 / FS], phase_poly=[[0.0] * 6])
    job = job_from_stations([st], n_chan=N // 2, n_frames=4, sub_start=first)
    y, d, v = fx.rotated_samples(job, 0, 0, 0, np.arange(4))
    Yf, _ = fx.station_spectra(job, 0, 0, 0, np.arange(4), frac=False, full_band=True)
    assert np.allclose(np.sum(np.abs(Yf) ** 2, axis=1), N * np.sum(np.abs(y) ** 2, axis=1),
                       rtol=1e-12)
    # zero phase polynomial: rotation is the identity
    y0, _, _ = fx.rotated_samples(job, 0, 0, 0, np.arange(4), rotate=False)
    assert np.array_equal(y, y0)
    # the integer delay of 3 samples reads the recording 3 samples later
    assert np.array_equal(y[0].real, _levels(codes[0, 3:3 + N]))
