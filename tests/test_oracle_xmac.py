"""Oracle pins: cross-multiply-accumulate and finalise (O9, O10).

Pinned by the brute-force lag-domain (XF) correlation, conjugate and Hermitian
symmetries, the flat white-noise autocorrelation level of the 4-level
quantiser, an exact phase rotation, and weights under bad frames.
"""
import numpy as np
import scipy.stats

from oracle import fx, xf
from synth import configs
from tests.helpers import rel_l2


def _small(**kw):
    base = dict(n_stations=3, n_subbands=2, n_pols=2, n_chan=16, C=4, n_frames=6)
    base.update(kw)
    return configs.small_job(**base)


def test_xf_equals_fx():
    job = _small()
    M, N = job.M, job.N
    V, W = fx.correlate(job)
    f = np.arange(job.n_frames)
    for sb in range(job.n_subbands):
        ys = [fx.rotated_samples(job, i // 2, sb, i % 2, f) for i in range(M)]
        for i in range(M):
            for j in range(i, M):
                yi, di, vi = ys[i]
                yj, dj, vj = ys[j]
                acc = np.zeros(N // 2, complex)
                cnt = 0
                for fr in f:
                    if not (vi[fr] and vj[fr]):
                        continue
                    k = np.arange(N // 2)
                    x = xf.xf_frame(yi[fr], yj[fr])[:N // 2]
                    acc += x * np.exp(2j * np.pi * k * (di[fr] - dj[fr]) / N)
                    cnt += 1
                bl = fx.baseline_index(i, j, M)
                assert W[sb, bl] == cnt > 0
                assert rel_l2(V[sb, bl], acc / cnt) < 1e-12


def test_conjugate_symmetry_under_input_swap():
    job = _small(n_pols=1, n_subbands=1, C=1)
    V, _ = fx.correlate(job)
    rev = configs.small_job(n_stations=3, n_subbands=1, n_pols=1, n_chan=16, C=1, n_frames=6)
    rev.stations = job.stations[::-1]
    Vr, _ = fx.correlate(rev)
    M = job.M
    for i in range(M):
        for j in range(i, M):
            a = V[0, fx.baseline_index(i, j, M)]
            b = Vr[0, fx.baseline_index(M - 1 - j, M - 1 - i, M)]
            assert np.allclose(a, np.conj(b), rtol=0, atol=1e-12 * np.abs(a).max())


def test_autos_real_nonnegative_and_cross_pol_complex():
    job = _small()
    V, _ = fx.correlate(job)
    M = job.M
    for i in range(M):
        a = V[:, fx.baseline_index(i, i, M)]
        assert np.all(a.imag == 0.0) and np.all(a.real >= 0)
    # p != q autos of one station are genuinely complex
    assert np.any(V[:, fx.baseline_index(0, 1, M)].imag != 0)


def test_full_band_hermitian_without_rotation():
    job = _small(n_chan=32, n_frames=5)
    V, _ = fx.correlate(job, rotate=False, full_band=True)
    N = job.N
    k = np.array([k for k in range(1, N) if k != N // 2])   # Nyquist has no signed frequency
    assert np.max(np.abs(V[..., N - k] - np.conj(V[..., k]))) < 1e-12 * np.max(np.abs(V))


def test_white_noise_autos_flat_at_quantiser_power():
    job = configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=256, C=1,
                            n_frames=300, seed=21)
    V, W = fx.correlate(job)
    p0 = scipy.stats.norm.cdf(-0.9816)
    Eq2 = 2 * p0 * fx.LEVELS[3] ** 2 + (1 - 2 * p0) * 1.0
    assert abs(Eq2 - 4.30481) < 1e-4
    E = job.N * Eq2                                    # 2204.1 at N = 512
    for s in range(2):
        A = V[0, fx.baseline_index(s, s, 2)].real
        w = W[0, fx.baseline_index(s, s, 2)]
        # per-channel estimate scatters by ~E/sqrt(W) (2-bit data is not exactly Gaussian)
        assert abs(A.mean() - E) < 4 * E / np.sqrt(w * A.size)
        assert 0.8 < A.std() / (E / np.sqrt(w)) < 1.25
        # no slope across the band
        k = np.arange(A.size)
        slope = np.polyfit(k, A / E, 1)[0] * A.size
        assert abs(slope) < 6 / np.sqrt(w * A.size) * np.sqrt(12)


def test_constant_phase_rotates_visibility_exactly():
    job = configs.small_job(n_stations=3, n_subbands=1, n_pols=1, n_chan=32, C=1,
                            n_frames=8, realistic=False)
    V0, _ = fx.correlate(job)
    c = [0.1, 0.37, -0.2]
    for s, st in enumerate(job.stations):
        st.phase_poly = np.array([[c[s], 0, 0, 0, 0, 0]], dtype=float)
    V1, _ = fx.correlate(job)
    for i in range(3):
        for j in range(i, 3):
            bl = fx.baseline_index(i, j, 3)
            rot = np.exp(2j * np.pi * (c[i] - c[j]))
            assert np.allclose(V1[0, bl], V0[0, bl] * rot, rtol=1e-12, atol=1e-9)


def test_weights_drop_frames_with_bad_sync():
    job = configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=64, C=1,
                            n_frames=900, realistic=False)
    V0, W0 = fx.correlate(job)
    st = job.stations[1]
    st.frames = st.frames.clone()
    st.frames[1, 0] = 0                                # second recording frame: bad sync
    V1, W1 = fx.correlate(job)
    n_int, _ = fx.frame_delays(st.delay_poly, job.sub_start, job.N, job.fs_hz,
                               np.arange(job.n_frames))
    base = job.sub_start + np.arange(job.n_frames) * job.N + n_int - st.first_sample
    hit = (base + job.N - 1 >= 40000) & (base < 80000)
    assert W1[0, 0] == W0[0, 0]
    assert W1[0, 1] == W0[0, 1] - hit.sum()
    assert W1[0, 2] == W0[0, 2] - hit.sum()
    keep = np.nonzero(~hit)[0]
    Vk, Wk = fx.correlate(job, frames=keep)
    assert np.array_equal(Wk[0, 1:], W1[0, 1:])
    assert rel_l2(V1[0, 1:], Vk[0, 1:]) < 1e-12
