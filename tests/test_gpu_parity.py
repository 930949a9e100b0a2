"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar: bit-exact for the integer delay, fractional delay, validity and 2-bit
unpack; relative L2 error over channels <= 1e-5 per baseline and subband for
visibilities (autos included); fringe phase at frame centres within 1e-8 turns.
"""
import zlib

import numpy as np
import pytest
import torch

from oracle import fx
from synth import configs
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def xc():
    from paper_1502_06894_amd import xcorr
    return xcorr


@pytest.fixture(scope="module")
def corr(xc):
    return xc.Correlator(0)


def _on_gpu(xc, job):
    return xc.job_to_device(job)


def _oracle_delays(job):
    F = np.arange(job.n_frames)
    out = []
    for st in job.stations:
        w = fx.as_words(st.frames)
        n_int, d = fx.frame_delays(st.delay_poly, job.sub_start, job.N, job.fs_hz, F)
        base, valid = fx.frame_valid(w, job.n_streams, st.first_sample, job.sub_start, job.N, F,
                                     n_int)
        out.append((n_int, d, valid))
    return out


def _jobs_for_delays():
    return [
        configs.small_job(n_stations=3, n_subbands=2, n_pols=2, n_chan=128, C=4, n_frames=300),
        configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=8192, C=1, n_frames=40,
                          seed=3),
        configs.c2_job(n_frames=700, n_subbands=2, n_stations=4),
    ]


@pytest.mark.parametrize("ji", range(3))
def test_delays_bit_exact(xc, corr, ji):
    job = _jobs_for_delays()[ji]
    ref = _oracle_delays(job)
    _on_gpu(xc, job)
    got = corr.debug_delays(job, frames_per_block=64)
    for s, (n_int, d, valid) in enumerate(ref):
        assert np.array_equal(got["n_int"][s], n_int), s
        assert np.array_equal(got["d"][s], d), s                      # bit-exact doubles
        assert np.array_equal(got["valid"][s], valid), s
        for sb in range(job.n_subbands):
            st = job.stations[s]
            pp = None if st.phase_poly is None else st.phase_poly[sb]
            f = np.arange(job.n_frames)
            ph = fx.fringe_phase(st.delay_poly, pp, job.lo_hz[sb], job.sub_start, job.N,
                                 job.fs_hz, f)[:, job.N // 2]
            err = (got["phi0"][s, sb] - ph + 0.5) % 1.0 - 0.5
            assert np.max(np.abs(err)) < 1e-8, (s, sb)


def test_unpack_bit_exact(xc, corr):
    rng = np.random.default_rng(1)
    for C, P, nsb in [(1, 1, 1), (2, 1, 2), (4, 2, 2), (8, 2, 4), (16, 2, 8)]:
        job = configs.small_job(n_stations=2, n_subbands=nsb, n_pols=P, n_chan=1024, C=C,
                                n_frames=60, seed=C)
        words = [fx.as_words(st.frames) for st in job.stations]
        _on_gpu(xc, job)
        for _ in range(6):
            s = int(rng.integers(0, 2))
            inp = int(rng.integers(0, nsb * P))
            f = int(rng.integers(0, job.n_frames))
            got = corr.debug_unpack(job, s, inp, f)
            y, _, valid = fx.rotated_samples(job, s, inp // P, inp % P, np.array([f]),
                                             rotate=False, words=words[s])
            want = y[0].real.astype(np.float32) if valid[0] else np.zeros(job.N, np.float32)
            assert np.array_equal(got, want), (C, s, inp, f)


@pytest.mark.parametrize("n_chan,C", [(128, 1), (256, 2), (1024, 16), (4096, 4), (8192, 8),
                                       (16384, 2)])
def test_spectra_parity(xc, corr, n_chan, C):
    P, nsb = (2, 2) if C >= 4 else (1, 1)
    job = configs.small_job(n_stations=2, n_subbands=nsb, n_pols=P, n_chan=n_chan, C=C,
                            n_frames=12, seed=n_chan)
    refs = {}
    for s in range(2):
        for sb in range(nsb):
            for p in range(P):
                refs[(s, sb, p)] = fx.station_spectra(job, s, sb, p, np.arange(12))[0]
    _on_gpu(xc, job)
    spec = corr.debug_spectra(job, 0, 12).cpu().numpy()          # [nsb, n, M, n_chan]
    for (s, sb, p), Y in refs.items():
        got = spec[sb, :, s * P + p, :]
        assert rel_l2(got, Y) < 3e-6, (s, sb, p)


@pytest.mark.parametrize("n_chan,C", [(256, 2), (1024, 16), (4096, 4), (8192, 8)])
def test_split_twiddles_parity(xc, corr, n_chan, C):
    """F-stage variant 5 (last-pass twiddles as products of two table entries):
    spectra within the F stage's bound of the oracle, visibilities within TOL."""
    P, nsb = (2, 2) if C >= 4 else (1, 1)
    job = configs.small_job(n_stations=3, n_subbands=nsb, n_pols=P, n_chan=n_chan, C=C,
                            n_frames=9, seed=n_chan + 7)
    V, W = fx.correlate(job, threads=8)
    _on_gpu(xc, job)
    try:
        corr.set_tuning(fstage_waves_per_simd=5)
        spec = corr.debug_spectra(job, 0, 9).cpu().numpy()
        vis, w = corr.correlate(job)
        vis = vis.cpu().numpy()
    finally:
        corr.set_tuning(fstage_waves_per_simd=0)
    for s in range(3):
        for sb in range(nsb):
            for p in range(P):
                Y = fx.station_spectra(job, s, sb, p, np.arange(9))[0]
                assert rel_l2(spec[sb, :, s * P + p, :], Y) < 3e-6, (s, sb, p)
    assert rel_l2(vis, V) < TOL


@pytest.mark.parametrize("n_chan,C,nsb,P,variant", [
    (1024, 16, 3, 2, 7),     # six inputs: a group of four and one of two
    (128, 4, 1, 1, 7),       # one input; 16 frames per workgroup
    (4096, 8, 5, 1, 0),      # the default at N = 8192 (lean): groups of four and one
    (8192, 16, 9, 1, 0),     # the default at N = 16384: groups 4 + 4 + 1
    (2048, 4, 2, 2, 7),      # lean at N = 4096, four inputs: one group
    (4096, 8, 5, 1, 1),      # one task per station and frame group at N = 8192
], ids=["lean2048_6in", "lean256_1in", "default8192_5in", "default16384_9in", "lean4096_4in",
        "classic8192"])
def test_fstage_task_shapes_parity(xc, corr, n_chan, C, nsb, P, variant):
    """F-stage task shapes (one task per station and frame group, or the lean
    tasks over groups of up to four inputs with packed codes): spectra within
    the F stage's bound of the oracle for every input, visibilities within TOL."""
    job = configs.small_job(n_stations=3, n_subbands=nsb, n_pols=P, n_chan=n_chan, C=C,
                            n_frames=7, seed=n_chan + 3 * nsb + P)
    V, W = fx.correlate(job, threads=8)
    _on_gpu(xc, job)
    try:
        corr.set_tuning(fstage_waves_per_simd=variant)
        spec = corr.debug_spectra(job, 0, 7).cpu().numpy()
        vis, w = corr.correlate(job)
        vis = vis.cpu().numpy()
    finally:
        corr.set_tuning(fstage_waves_per_simd=0)
    for s in range(3):
        for sb in range(nsb):
            for p in range(P):
                Y = fx.station_spectra(job, s, sb, p, np.arange(7))[0]
                assert rel_l2(spec[sb, :, s * P + p, :], Y) < 3e-6, (s, sb, p)
    assert np.array_equal(w.cpu().numpy(), W.astype(np.float32))
    for sb in range(nsb):
        for bl in range(job.n_baselines):
            assert rel_l2(vis[sb, bl], V[sb, bl]) < TOL, (sb, bl)


VIS_CASES = [
    # name, small_job kwargs, frames_per_block
    ("c1like", dict(n_stations=2, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=300), 0),
    ("ragged", dict(n_stations=3, n_subbands=2, n_pols=2, n_chan=128, C=4, n_frames=37), 16),
    ("c2like", dict(n_stations=4, n_subbands=8, n_pols=2, n_chan=1024, C=16, n_frames=40), 0),
    ("c4like", dict(n_stations=5, n_subbands=4, n_pols=1, n_chan=4096, C=4, n_frames=12), 0),
    ("big_n", dict(n_stations=2, n_subbands=1, n_pols=1, n_chan=8192, C=2, n_frames=6), 0),
    ("matched", dict(n_stations=6, n_subbands=2, n_pols=1, n_chan=512, C=8, n_frames=50,
                     realistic=False), 0),
    ("one_frame", dict(n_stations=2, n_subbands=1, n_pols=2, n_chan=2048, C=2, n_frames=1), 0),
    ("m_not_mult4", dict(n_stations=7, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=20), 8),
    ("splits", dict(n_stations=3, n_subbands=1, n_pols=2, n_chan=128, C=2, n_frames=700), 600),
    ("m32", dict(n_stations=32, n_subbands=1, n_pols=1, n_chan=128, C=1, n_frames=30), 0),
    ("n32768", dict(n_stations=3, n_subbands=1, n_pols=2, n_chan=16384, C=2, n_frames=5), 0),
    ("n32768_blocks", dict(n_stations=2, n_subbands=2, n_pols=1, n_chan=16384, C=4, n_frames=7),
     3),
]


@pytest.mark.parametrize("name,kw,fpb", VIS_CASES, ids=[c[0] for c in VIS_CASES])
def test_visibility_parity(xc, corr, name, kw, fpb):
    job = configs.small_job(**kw, seed=zlib.crc32(name.encode()) % 1000)
    V, W = fx.correlate(job, threads=8)
    _on_gpu(xc, job)
    vis, w = corr.correlate(job, frames_per_block=fpb)
    torch.cuda.synchronize()
    vis, w = vis.cpu().numpy(), w.cpu().numpy()
    assert np.array_equal(w, W.astype(np.float32))
    assert rel_l2(vis, V) < TOL, name


@pytest.mark.parametrize("tau2", [3e-8, 1.6e-3])
def test_perigee_acceleration_parity(xc, corr, tau2):
    """A space station near perigee: delay rate 3e-5 s/s and delay acceleration tau''
    of 3e-8 s/s^2 (gravity-class) and 1.6e-3 s/s^2 (a stress case whose quadratic
    fringe phase reaches ~0.1 rad across an N = 4096 frame): the per-frame phase
    Taylor terms and the second-order phasor recurrence match the oracle's per-sample
    long-double phase."""
    from synth import shape
    fs, n_chan, t0 = configs.FS_16MHZ, 2048, configs.SUB_START_S
    ground = [0.011, -2e-6, 0.0]
    # space(t) = 0.08 + 3e-5 (t - t0) + tau2 / 2 (t - t0)^2, expanded about t = 0
    space = [0.08 - 3e-5 * t0 + 0.5 * tau2 * t0 * t0, 3e-5 - tau2 * t0, 0.5 * tau2]
    job = shape.build_job(n_stations=2, n_subbands=2, n_pols=1, n_chan=n_chan, C=2, fs=fs,
                          lo_hz=[configs.LO0_HZ, configs.LO0_HZ + 16e6],
                          sub_start=int(t0 * fs), n_frames=40, delay_polys=[ground, space],
                          shifts=[0, 0], phase_zero=False, seed=91, margin=4096)
    V, W = fx.correlate(job, threads=8)
    _on_gpu(xc, job)
    vis, w = corr.correlate(job)
    assert np.array_equal(w.cpu().numpy(), W.astype(np.float32))
    assert rel_l2(vis.cpu().numpy(), V) < TOL


@pytest.mark.parametrize("rate,n_chan", [(3e-5, 2048), (3e-4, 512), (3e-5, 8192)])
def test_drift_correction_parity(xc, corr, rate, n_chan):
    """Intra-frame delay-drift correction (O11) on the space station: spectra and
    visibilities against the oracle, and the correction is not a no-op."""
    import dataclasses
    from synth import shape
    fs, t0 = configs.FS_16MHZ, configs.SUB_START_S
    ground = [0.011, -2e-6, 0.0]
    space = [0.08 - rate * t0, rate, 0.0]
    job = shape.build_job(n_stations=2, n_subbands=2, n_pols=1, n_chan=n_chan, C=2, fs=fs,
                          lo_hz=[configs.LO0_HZ, configs.LO0_HZ + 16e6],
                          sub_start=int(t0 * fs), n_frames=12, delay_polys=[ground, space],
                          shifts=[0, 0], phase_zero=False, seed=93, margin=4096)
    off = job
    job = dataclasses.replace(job, stations=[job.stations[0],
                                             dataclasses.replace(job.stations[1], rate_correct=True)])
    Y = fx.station_spectra(job, 1, 1, 0, np.arange(12))[0]
    Y0 = fx.station_spectra(off, 1, 1, 0, np.arange(12))[0]
    assert rel_l2(Y0, Y) > 1e-4 * rate / 3e-5          # the correction changes the spectra
    V, W = fx.correlate(job, threads=8)
    _on_gpu(xc, job)
    spec = corr.debug_spectra(job, 0, 12).cpu().numpy()
    assert rel_l2(spec[1, :, 1, :], Y) < 3e-6
    assert rel_l2(spec[1, :, 0, :], fx.station_spectra(job, 0, 1, 0, np.arange(12))[0]) < 3e-6
    vis, w = corr.correlate(job)
    assert np.array_equal(w.cpu().numpy(), W.astype(np.float32))
    assert rel_l2(vis.cpu().numpy(), V) < TOL


def test_drift_correction_limits(xc, corr):
    import dataclasses
    job = configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=8)
    job = dataclasses.replace(job, stations=[dataclasses.replace(job.stations[0], rate_correct=True),
                                             job.stations[1]])
    _on_gpu(xc, job)
    with pytest.raises(xc.XcError) as e:
        corr.correlate(job, precision=xc.XC_FP16_MFMA)
    assert e.value.code == xc.XC_E_INVAL


def test_bad_frames_and_out_of_buffer(xc, corr):
    job = configs.small_job(n_stations=3, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=400,
                            realistic=False, seed=5)
    st = job.stations[1]
    st.frames = st.frames.clone()
    st.frames[2, 0] = 0                                # bad sync in recording frame 2
    job.stations[2].frames = job.stations[2].frames[:-1].contiguous()   # last frames out of buffer
    V, W = fx.correlate(job, threads=8)
    assert W.min() < job.n_frames
    _on_gpu(xc, job)
    vis, w = corr.correlate(job)
    assert np.array_equal(w.cpu().numpy(), W.astype(np.float32))
    assert rel_l2(vis.cpu().numpy(), V) < TOL


def test_n32768_input_groups_and_invalid_frames(xc, corr):
    """N = 32768 (the folded FP32 F stage, tasks over groups of four inputs):
    six inputs per station (a group of four and one of two), a bad sync word
    on one station and the last FFT frame of another outside its recording."""
    job = configs.small_job(n_stations=3, n_subbands=3, n_pols=2, n_chan=16384, C=8, n_frames=6,
                            seed=41)
    job.stations[0].frames = job.stations[0].frames.clone()
    job.stations[0].frames[3, 0] = 0                   # bad sync in recording frame 3
    job.stations[2].frames = job.stations[2].frames[:-3].contiguous()   # the end is cut
    V, W = fx.correlate(job, threads=8)
    assert W.min() < job.n_frames - 1 and W.max() == job.n_frames
    _on_gpu(xc, job)
    vis, w = corr.correlate(job)
    assert np.array_equal(w.cpu().numpy(), W.astype(np.float32))
    vis = vis.cpu().numpy()
    for sb in range(job.n_subbands):
        for bl in range(job.n_baselines):
            if W[sb, bl] > 0:
                assert rel_l2(vis[sb, bl], V[sb, bl]) < TOL, (sb, bl)


def test_invalid_frames_across_weight_chunks(xc, corr):
    """One 5000-frame block (the default for a job this small), so the pair
    weights are counted over three 2048-frame chunks; bad sync words and the
    end of a recording fall in different chunks."""
    job = configs.small_job(n_stations=3, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=5000,
                            realistic=False, seed=11)
    for s_, m in ((1, 10), (0, 45)):                   # FFT frames ~780 and ~3500
        job.stations[s_].frames = job.stations[s_].frames.clone()
        job.stations[s_].frames[m, 0] = 0
    job.stations[2].frames = job.stations[2].frames[:-2].contiguous()   # the last frames
    V, W = fx.correlate(job, threads=8)
    assert W.min() < job.n_frames - 100
    _on_gpu(xc, job)
    vis, w = corr.correlate(job)
    assert np.array_equal(w.cpu().numpy(), W.astype(np.float32))
    assert rel_l2(vis.cpu().numpy(), V) < TOL
    vis2, w2 = corr.correlate(job, frames_per_block=2048)
    assert torch.equal(w, w2)
    assert rel_l2(vis2.cpu().numpy(), V) < TOL


def test_ingest_mask_and_supplied_mask(xc, corr):
    job = configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=200,
                            realistic=False, seed=8)
    job.stations[0].frames = job.stations[0].frames.clone()
    job.stations[0].frames[1, 0] = 123
    want = fx.sync_ok(fx.as_words(job.stations[0].frames))
    _on_gpu(xc, job)
    ok = corr.ingest(job.stations[0].frames)
    assert np.array_equal(ok.cpu().numpy().astype(bool), want)
    oks = [corr.ingest(st.frames) for st in job.stations]
    v1, w1 = corr.correlate(job)
    v2, w2 = corr.correlate(job, frame_ok=oks)
    assert torch.equal(v1, v2) and torch.equal(w1, w2)


def test_error_codes(xc, corr):
    job = configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=10)
    _on_gpu(xc, job)
    with pytest.raises(xc.XcError) as e:
        corr.correlate(job, workspace=torch.empty(1024, dtype=torch.uint8, device="cuda"))
    assert e.value.code == xc.XC_E_NOMEM
    job.stations[0].poly_span = (0.0, 10.0)
    with pytest.raises(xc.XcError) as e:
        corr.correlate(job)
    assert e.value.code == xc.XC_E_RANGE


def test_deterministic_repeat(xc, corr):
    job = configs.small_job(n_stations=4, n_subbands=2, n_pols=2, n_chan=512, C=4, n_frames=90)
    _on_gpu(xc, job)
    a = corr.correlate(job)[0].clone()
    for _ in range(3):
        assert torch.equal(corr.correlate(job)[0], a)


def test_block_overlap_bit_identical(xc, corr):
    """F of block b + 1 beside X of block b on a second stream: same visibilities bit for bit,
    including a ragged last block."""
    job = configs.small_job(n_stations=4, n_subbands=2, n_pols=2, n_chan=256, C=4, n_frames=300)
    V, W = fx.correlate(job, threads=8)
    _on_gpu(xc, job)
    try:
        corr.set_tuning(block_overlap=1)
        ref, w0 = corr.correlate(job, frames_per_block=64)
        assert rel_l2(ref.cpu().numpy(), V) < TOL
        corr.set_tuning(block_overlap=2)
        big = corr.workspace_bytes(job, frames_per_block=64)
        corr.set_tuning(block_overlap=1)
        assert big > corr.workspace_bytes(job, frames_per_block=64)   # two block buffers
        corr.set_tuning(block_overlap=2)
        for _ in range(2):
            vis, w = corr.correlate(job, frames_per_block=64)
            assert torch.equal(vis, ref) and torch.equal(w, w0)
    finally:
        corr.set_tuning(block_overlap=0)


MATRIX_CASES = [
    # name, small_job kwargs, frames_per_block: every input-group count 1..8
    # (one and two tile parts per channel block), ragged frame counts and
    # several slots
    ("mg1", dict(n_stations=2, n_subbands=1, n_pols=1, n_chan=128, C=1, n_frames=9), 0),
    ("one_input", dict(n_stations=1, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=11), 0),
    ("mg2", dict(n_stations=3, n_subbands=1, n_pols=2, n_chan=256, C=2, n_frames=23), 0),
    ("mg3", dict(n_stations=6, n_subbands=2, n_pols=2, n_chan=128, C=4, n_frames=41), 0),
    ("mg4", dict(n_stations=16, n_subbands=1, n_pols=1, n_chan=128, C=1, n_frames=13), 0),
    ("mg5_c2like", dict(n_stations=10, n_subbands=2, n_pols=2, n_chan=128, C=4, n_frames=37),
     16),
    ("mg6", dict(n_stations=23, n_subbands=1, n_pols=1, n_chan=128, C=1, n_frames=30), 0),
    ("mg7", dict(n_stations=14, n_subbands=1, n_pols=2, n_chan=128, C=2, n_frames=19), 0),
    ("mg8_slots", dict(n_stations=32, n_subbands=1, n_pols=1, n_chan=128, C=1, n_frames=700),
     600),
]


@pytest.mark.parametrize("staging", ["matrix", "matrix_ring"])
@pytest.mark.parametrize("name,kw,fpb", MATRIX_CASES, ids=[c[0] for c in MATRIX_CASES])
def test_matrix_core_x_stage(xc, corr, name, kw, fpb, staging):
    """FP32 X stage on the matrix cores, operands loaded per wave (matrix) or
    fed through the LDS ring (matrix_ring): each 4x4x1 block element is a fused
    multiply-add with one rounding, issued in the vector kernels' order, so the
    visibilities equal the vector ring's bit for bit (and the oracle's within
    the FP32 tolerance)."""
    job = configs.small_job(**kw, seed=zlib.crc32(name.encode()) % 1000)
    V, W = fx.correlate(job, threads=8)
    _on_gpu(xc, job)
    fb = {"matrix": xc.XMAC_MATRIX, "matrix_ring": xc.XMAC_MATRIX_RING}[staging]
    try:
        corr.set_tuning(xmac_frames_per_stage=8)   # the vector ring
        vec, w0 = corr.correlate(job, frames_per_block=fpb)
        corr.set_tuning(xmac_frames_per_stage=fb)
        mat, w1 = corr.correlate(job, frames_per_block=fpb)
        torch.cuda.synchronize()
    finally:
        corr.set_tuning(xmac_frames_per_stage=0)
    assert torch.equal(w0, w1)
    assert torch.equal(vec, mat), name
    assert rel_l2(mat.cpu().numpy(), V) < TOL, name


def test_x_kernels_slice_blocks_alike(xc, corr):
    """A block large enough for the X stage to pick its slice count by whole
    rounds of workgroups (2100 frames, 20 inputs, 8 subbands, 1024 channels:
    four slices of 525 frames rather than three of 700): the ring-fed matrix
    kernel (the default), the vector ring, the per-wave matrix kernel and the
    register-staged kernel all cut it alike and give the same bits."""
    job = configs.small_job("cuda", n_stations=10, n_subbands=8, n_pols=2, n_chan=1024, C=16,
                            n_frames=2100, seed=77, realistic=True)
    outs = {}
    try:
        for fb in (0, 8, xc.XMAC_MATRIX, 2):
            corr.set_tuning(xmac_frames_per_stage=fb)
            outs[fb] = corr.correlate(job, frames_per_block=2100)
        torch.cuda.synchronize()
    finally:
        corr.set_tuning(xmac_frames_per_stage=0)
    v0, w0 = outs[0]
    for fb, (v, w) in outs.items():
        assert torch.equal(w, w0) and torch.equal(v, v0), fb


def test_tuning_variants_bit_identical(xc, corr):
    """Launch-shape variants change speed only: visibilities must be bit-identical
    (F-stage variants 1, 3, 4 and the pol-sharing 2 (the dual-pol default) and 8
    included)."""
    job = configs.small_job(n_stations=5, n_subbands=2, n_pols=2, n_chan=256, C=4, n_frames=300)
    V, W = fx.correlate(job, threads=8)
    _on_gpu(xc, job)
    ref = None
    try:
        for tune in [dict(), dict(xmac_frames_per_stage=8), dict(xmac_frames_per_stage=8, xmac_tiles_per_wg=2),
                     dict(xmac_frames_per_stage=1), dict(xmac_frames_per_stage=2),
                     dict(xmac_frames_per_stage=4, xmac_channels_per_wg=16),
                     dict(xmac_frames_per_stage=1, xmac_channels_per_wg=32),
                     dict(xmac_frames_per_stage=1, xmac_tiles_per_wg=1),
                     dict(xmac_frames_per_stage=1, xmac_tiles_per_wg=3, xmac_channels_per_wg=16),
                     dict(xmac_frames_per_stage=3),
                     dict(xmac_frames_per_stage=5),
                     dict(fstage_waves_per_simd=1), dict(fstage_waves_per_simd=2),
                     dict(fstage_waves_per_simd=3),
                     dict(fstage_waves_per_simd=4), dict(fstage_waves_per_simd=8)]:
            base = dict(fstage_waves_per_simd=0, xmac_frames_per_stage=0, xmac_channels_per_wg=0,
                        xmac_tiles_per_wg=0)
            base.update(tune)
            corr.set_tuning(**base)
            vis, w = corr.correlate(job, frames_per_block=300)
            vis = vis.cpu()
            if ref is None:
                ref = vis
                assert rel_l2(vis.numpy(), V) < TOL
            assert torch.equal(vis, ref), tune
    finally:
        corr.set_tuning(fstage_waves_per_simd=0, xmac_frames_per_stage=0, xmac_channels_per_wg=0,
                        xmac_tiles_per_wg=0)
