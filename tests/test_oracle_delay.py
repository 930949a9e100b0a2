"""Oracle pins: delay model and frame validity (O1-O4).

Pinned by closed forms (constant and linear delays), exact rational
arithmetic, and hand-placed bad frames.
"""
from fractions import Fraction

import numpy as np

from oracle import fx
from synth import configs
from tests.helpers import station_from_codes

FS = 32e6


def test_constant_delay_gives_integer_shift():
    f = np.arange(200)
    for k in [0, 1, 137, -2000, 12_812_345]:
        n_int, d = fx.frame_delays([k / FS, 0, 0, 0, 0, 0], 1_184_000_000, 512, FS, f)
        assert np.all(n_int == k)
        assert np.all(np.abs(d) < 1e-6)


def test_one_sample_more_delay_shifts_by_one():
    f = np.arange(500)
    p = list(configs.SPACE_C1)
    n0, d0 = fx.frame_delays(p, 1_184_000_000, 2048, FS, f)
    p[0] += 1.0 / FS
    n1, d1 = fx.frame_delays(p, 1_184_000_000, 2048, FS, f)
    assert np.all(n1 - n0 == 1)
    assert np.max(np.abs(d1 - d0)) < 1e-7


def test_linear_delay_closed_form_uses_frame_centre():
    # tau(t) = t / 64 (exact binary coefficient): D = (j0 + f N + N/2) / 64.
    # j0 = 64 m + 16 puts D at an integer + 0.25, so n_int and d are fixed exactly.
    N, m = 512, 18_500_000
    j0 = 64 * m + 16
    f = np.arange(300)
    n_int, d = fx.frame_delays([0.0, 1.0 / 64.0], j0, N, FS, f)
    assert np.all(n_int == m + 8 * f + 4)
    assert np.all(np.abs(d - 0.25) < 1e-6)


def test_horner_against_exact_rationals():
    rng = np.random.default_rng(5)
    for trial in range(40):
        c = [float(x) for x in np.array(configs.SPACE_C1) * rng.uniform(0.5, 1.5, 6)]
        t = float(rng.uniform(0, 120))
        got = fx.horner(c, np.array([t]))[0]
        exact = sum(Fraction(ck) * Fraction(t) ** k for k, ck in enumerate(c))
        scale = sum(abs(Fraction(ck) * Fraction(t) ** k) for k, ck in enumerate(c))
        assert abs(Fraction(got) - exact) <= 8 * Fraction(2.0 ** -53) * scale, trial
        # a dropped or mis-indexed term would be off by far more than rounding
        D = exact * Fraction(FS)
        n_int, d = fx.frame_delays(c, 0, 2, FS, np.array([0]))
        # frame_delays evaluates at t_mid = 1 / fs; redo the exact value there
        tm = Fraction(1) / Fraction(FS)
        De = sum(Fraction(ck) * tm ** k for k, ck in enumerate(c)) * Fraction(FS)
        assert n_int[0] == int(np.floor(float(De) + 0.5))
        assert abs(d[0] - float(De - n_int[0])) < 1e-6


def test_validity_edges_and_sync():
    C, N = 1, 512
    spf = 40000
    first = 1_000_000
    codes = np.full((1, 4 * spf), 2)
    st = station_from_codes(codes, C, first, [0.0] * 6)
    w = fx.as_words(st.frames)
    # window starts: frame f reads [sub_start + f N, ...) with zero delay
    sub_start = first - 2 * N                     # first two frames start before the recording
    f = np.arange(4 * spf // N + 4)
    n_int = np.zeros_like(f)
    base, valid = fx.frame_valid(w, C, first, sub_start, N, f, n_int)
    assert list(valid[:3]) == [False, False, True]
    last_ok = (4 * spf + 2 * N) // N - 1          # last frame whose window ends inside
    assert valid[last_ok] and not valid[last_ok + 1]
    # a bad sync word invalidates exactly the frames whose windows touch that frame
    w2 = w.copy()
    w2[1, 0] = 0
    _, v2 = fx.frame_valid(w2, C, first, sub_start, N, f, n_int)
    touch = (base + N - 1 >= spf) & (base < 2 * spf)
    assert np.array_equal(v2, valid & ~touch)
