"""GPU: the MFMA X stage with FP16 / FP8 (e4m3) spectra against the FP64 oracle.

Each spectrum component is rounded once (after a power-of-two scale that
cannot overflow for these data), so |dY| <= u |Y| with u = 2^-11 (FP16) or
2^-4 (e4m3), and every product Y_i conj(Y_j) is off by at most
(2u + u^2)|Y_i||Y_j|.  Averaged over frames and bounded by Cauchy-Schwarz:
    |dV_ij[k]| <= (2u + u^2) sqrt(A_i[k] A_j[k])
with A the oracle's autocorrelations.  The test asserts that bound (10 %
slack for FP32 accumulation and the FP32 F stage) per baseline, subband and
channel, and prints the per-baseline error table.
"""
import numpy as np
import pytest
import torch

from oracle import fx
from synth import configs

pytestmark = pytest.mark.gpu

U = {"fp16": 2.0 ** -11, "fp8": 2.0 ** -4}


@pytest.fixture(scope="module")
def xc():
    from paper_1502_06894_amd import xcorr
    return xcorr


@pytest.fixture(scope="module")
def corr(xc):
    return xc.Correlator(0)


def _norm_err(vis, V, job):
    M = job.M
    worst = 0.0
    rows = []
    for sb in range(job.n_subbands):
        for i in range(M):
            for j in range(i, M):
                bl = fx.baseline_index(i, j, M)
                Ai = V[sb, fx.baseline_index(i, i, M)].real
                Aj = V[sb, fx.baseline_index(j, j, M)].real
                d = np.abs(vis[sb, bl] - V[sb, bl]) / np.sqrt(Ai * Aj)
                rel = np.linalg.norm(vis[sb, bl] - V[sb, bl]) / np.linalg.norm(V[sb, bl])
                worst = max(worst, float(d.max()))
                rows.append((sb, i, j, float(d.max()), float(rel)))
    return worst, rows


def _c4_shaped():
    # the C4 geometry (32 stations, 64 Msps, N = 8192, 4096 channels) over 96 frames
    return configs.c4_job(n_frames=96, n_subbands=1)


@pytest.mark.parametrize("prec", ["fp16", "fp8"])
@pytest.mark.parametrize("kw", [
    dict(n_stations=32, n_subbands=2, n_pols=1, n_chan=512, C=4, n_frames=96, realistic=False),
    dict(n_stations=6, n_subbands=2, n_pols=2, n_chan=256, C=4, n_frames=75),
    None,
    dict(n_stations=4, n_subbands=5, n_pols=1, n_chan=4096, C=8, n_frames=24, realistic=False),
    dict(n_stations=3, n_subbands=2, n_pols=1, n_chan=16384, C=2, n_frames=5),
], ids=["m32", "dualpol", "c4shape", "lean_5in", "n32768"])
def test_mfma_precision_bound(xc, corr, prec, kw):
    job = _c4_shaped() if kw is None else configs.small_job(**kw, seed=17)
    V, W = fx.correlate(job, threads=8)
    xc.job_to_device(job)
    fpb = 64 if kw is not None else 0
    vis, w = corr.correlate(job, precision=xc.PRECISIONS[prec], frames_per_block=fpb)
    torch.cuda.synchronize()
    vis, w = vis.cpu().numpy(), w.cpu().numpy()
    assert np.array_equal(w, W.astype(np.float32))
    worst, rows = _norm_err(vis, V, job)
    u = U[prec]
    bound = 1.1 * (2 * u + u * u)
    rel = np.array([r[4] for r in rows])
    auto = np.array([r[3] for r in rows if r[1] == r[2]])
    cross = np.array([r[3] for r in rows if r[1] != r[2]])
    print(f"\n{prec} {job.M} inputs, {job.n_chan} channels: max |dV|/sqrt(AiAj) = {worst:.3e} "
          f"(bound {bound:.3e}); per baseline max over channels: autos median "
          f"{np.median(auto):.3e} max {auto.max():.3e}, crosses median {np.median(cross):.3e} "
          f"max {cross.max():.3e}; per-baseline relative L2: median {np.median(rel):.3e}, "
          f"max {rel.max():.3e}")
    assert worst <= bound


def _late_start(job, station, first_valid):
    """Cut the start of a station's recording so that its FFT frames before
    `first_valid` fall outside it (and frame `first_valid` stays inside)."""
    from synth import format as fmt
    st = job.stations[station]
    spf = fmt.samples_per_frame(job.n_streams)
    n_int, _ = fx.frame_delays(st.delay_poly, job.sub_start, job.N, job.fs_hz,
                               np.array([first_valid - 1, first_valid]))
    base = job.sub_start + np.array([first_valid - 1, first_valid]) * job.N + n_int - st.first_sample
    k = int(base[0]) // spf + 1               # recording frames to drop
    assert k * spf > base[0] and k * spf <= base[1]
    st.frames = st.frames[k:].contiguous()
    st.first_sample += k * spf


@pytest.mark.parametrize("prec", ["fp16", "fp8"])
def test_mfma_scales_from_valid_frames(xc, corr, prec):
    """Channel scales come from the pre-pass frames valid for each station:
    station 1's recording starts after the 64 scale frames and station 2's
    after 62 of them (two valid frames: too few for a per-channel estimate);
    both take the expected white-noise level.  Unscaled, the spectra of an
    N = 32768 frame (RMS ~375) would saturate e4m3 (max 448) on ~9 % of their
    components; scaled from two frames, a few of 16384 channels would."""
    job = configs.small_job(n_stations=3, n_subbands=1, n_pols=1, n_chan=16384, C=2,
                            n_frames=80, seed=23)
    _late_start(job, 1, 66)
    _late_start(job, 2, 62)
    V, W = fx.correlate(job, threads=8)
    assert W[0, fx.baseline_index(1, 1, 3)] == 14 and W[0, fx.baseline_index(2, 2, 3)] == 18
    xc.job_to_device(job)
    vis, w = corr.correlate(job, precision=xc.PRECISIONS[prec])
    torch.cuda.synchronize()
    vis, w = vis.cpu().numpy(), w.cpu().numpy()
    assert np.array_equal(w, W.astype(np.float32))
    worst, _ = _norm_err(vis, V, job)
    u = U[prec]
    print(f"\n{prec} late-start stations: max |dV|/sqrt(AiAj) = {worst:.3e}")
    assert worst <= 1.1 * (2 * u + u * u)


def test_mfma_rejects_more_than_32_inputs(xc, corr):
    job = configs.small_job(n_stations=17, n_subbands=1, n_pols=2, n_chan=128, C=2, n_frames=4)
    xc.job_to_device(job)
    with pytest.raises(xc.XcError) as e:
        corr.correlate(job, precision=xc.XC_FP16_MFMA)
    assert e.value.code == xc.XC_E_INVAL
