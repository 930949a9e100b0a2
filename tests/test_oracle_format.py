"""Oracle pins: recording format (A0, O5).

The packer in synth.format and the oracle's unpack_codes are independent
implementations of the repository's Mark5B-style layout; a round trip pins
both against each other, and a hand-assembled word pins them to the written
layout itself.
"""
import numpy as np
import pytest
import scipy.stats
import torch

from oracle import fx
from synth import format as fmt


@pytest.mark.parametrize("C", [1, 2, 4, 8, 16])
def test_pack_unpack_roundtrip(C):
    rng = np.random.default_rng(100 + C)
    spf = fmt.samples_per_frame(C)
    n = 3 * spf
    codes = rng.integers(0, 4, size=(C, n))
    frames = fmt.frame_codes(torch.from_numpy(codes), C, first_sample=12345, fs_hz=32e6,
                             station_id=3)
    w = fx.as_words(frames)
    assert w.shape == (3, 2504)
    for c in range(C):
        assert np.array_equal(fx.unpack_codes(w, C, c, np.arange(n)), codes[c])
    # unaligned windows, including ones that straddle a frame boundary
    for start in [1, spf - 5, spf - 1, spf, 2 * spf - 7, 17]:
        pos = start + np.arange(min(97, n - start))
        c = start % C
        assert np.array_equal(fx.unpack_codes(w, C, c, pos), codes[c, pos])


def test_hand_assembled_word():
    # C = 4: fields 0..3 are streams 0..3 at time 0, fields 4..7 streams 0..3 at time 1, ...
    word = 0
    expect = {}
    for j in range(16):
        code = (j * 7 + 1) % 4
        word |= code << (2 * j)
        expect[(j % 4, j // 4)] = code
    w = np.zeros((1, 2504), dtype=np.uint32)
    w[0, 0] = fmt.SYNC_WORD
    w[0, 4] = word
    for (stream, t), code in expect.items():
        assert fx.unpack_codes(w, 4, stream, np.array([t]))[0] == code
    # C = 1: field j is time j of the only stream; C = 16: field j is stream j at time 0
    for j in range(16):
        assert fx.unpack_codes(w, 1, 0, np.array([j]))[0] == (j * 7 + 1) % 4
        assert fx.unpack_codes(w, 16, j, np.array([0]))[0] == (j * 7 + 1) % 4


def test_headers():
    C, fs = 16, 32e6
    spf = fmt.samples_per_frame(C)
    first = 37 * 32_000_000 - 3 * spf
    h = fx.as_words(fmt.headers(6, C, first, fs, station_id=5))
    assert (h[:, 0] == 0xABADDEED).all()
    assert list(h[:, 2]) == [36, 36, 36, 37, 37, 37]
    assert list(h[:, 1] & 0x7FFF) == [12797, 12798, 12799, 0, 1, 2]
    assert (h[:, 1] >> 16 == 5).all()
    assert (h[:, 3] == 0).all()


def test_code_frequencies_and_levels():
    # optimum 4-level quantiser: P(code 0) = P(code 3) = Phi(-0.9816)
    g = torch.Generator().manual_seed(11)
    x = torch.randn(2_000_000, generator=g, dtype=torch.float64)
    codes = fmt.quantise(x).numpy()
    freq = np.bincount(codes, minlength=4) / codes.size
    p0 = scipy.stats.norm.cdf(-0.9816)
    expect = np.array([p0, 0.5 - p0, 0.5 - p0, p0])
    assert np.allclose(expect, [0.1631, 0.3369, 0.3369, 0.1631], atol=1e-4)
    sig = np.sqrt(expect * (1 - expect) / codes.size)
    assert np.all(np.abs(freq - expect) < 5 * sig)
    # levels: offset binary, symmetric, the outer level is the float32 3.3359
    assert list(fx.LEVELS[:3]) == [float(np.float32(-3.3359)), -1.0, 1.0]
    assert fx.LEVELS[3] == -fx.LEVELS[0] == 3.335900068283081


def test_sync_mask():
    codes = torch.zeros(1, 4 * 40000, dtype=torch.int64)
    fr = fmt.frame_codes(codes, 1, 0, 32e6, 0)
    fr[2, 0] = 0
    assert list(fx.sync_ok(fx.as_words(fr))) == [True, True, False, True]
