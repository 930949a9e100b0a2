"""GPU: batches (the fused executor, lanes, hipGraph capture/replay) and the
autotuner.

A batch must reproduce each job's stand-alone result bit for bit: the fused
executor runs each job's blocks through the same arithmetic (one launch over
the blocks of many jobs of one FFT length per round), the lane executor the
same kernels concurrently; for any lane count and on graph replay.  A few jobs
are also checked against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from oracle import fx
from synth import configs
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xc():
    from paper_1502_06894_amd import xcorr
    return xcorr


@pytest.fixture(scope="module")
def corr(xc):
    return xc.Correlator(0)


def _jobs(xc):
    rng = np.random.default_rng(2024)
    jobs = []
    for i in range(12):
        P = int(rng.integers(1, 3))
        nsb = int(rng.integers(1, 5))
        C = int(2 ** rng.integers(int(np.ceil(np.log2(nsb * P))), 5))
        jobs.append(configs.small_job(n_stations=int(rng.integers(2, 9)), n_subbands=nsb, n_pols=P,
                                      n_chan=int(2 ** rng.integers(7, 12)), C=C,
                                      n_frames=int(rng.integers(1, 120)), seed=100 + i,
                                      realistic=bool(i % 2)))
    return jobs


@pytest.fixture(scope="module")
def batch(xc, corr):
    jobs = _jobs(xc)
    refs = []
    for j in jobs:
        xc.job_to_device(j)
        v, w = corr.correlate(j)
        refs.append((v.clone(), w.clone()))
    torch.cuda.synchronize()
    return jobs, refs


def test_batch_matches_single_jobs_bitwise(xc, corr, batch):
    jobs, refs = batch
    for lanes_only in (False, True):
        for lanes in (1, 3, 8):
            outs = corr.correlate_batch(jobs, n_lanes=lanes, lanes_only=lanes_only)
            torch.cuda.synchronize()
            for (v, w), (rv, rw) in zip(outs, refs):
                assert torch.equal(v, rv) and torch.equal(w, rw), (lanes_only, lanes)


def _fused_mix(xc):
    """Jobs for the fused executor's corner cases: several FFT lengths (the
    lean F stage at 8192 and 16384 points), single and dual pol, input counts
    of several tile shapes in one length, two jobs on the same recordings
    (one mask each), a bad sync word and a recording cut short; plus jobs it
    hands to single-job runs (16384 channels, FP16 precision, drift correction)."""
    import dataclasses
    rng = np.random.default_rng(404)
    jobs, precs = [], []
    for i, (S, nsb, P, n_chan, C, F) in enumerate([
            (3, 2, 1, 256, 2, 300), (9, 1, 1, 256, 1, 140), (2, 3, 2, 256, 8, 200),
            (5, 2, 1, 4096, 2, 40), (4, 5, 1, 8192, 8, 9), (3, 2, 1, 4096, 2, 70),
            (6, 1, 2, 1024, 2, 90), (2, 1, 1, 16384, 1, 4), (3, 1, 1, 512, 1, 50)]):
        jobs.append(configs.small_job(n_stations=S, n_subbands=nsb, n_pols=P, n_chan=n_chan, C=C,
                                      n_frames=F, seed=500 + i, realistic=bool(i % 2)))
        precs.append(xc.XC_FP32)
    jobs[1].stations[2].frames = jobs[1].stations[2].frames.clone()
    jobs[1].stations[2].frames[1, 0] = 0                      # bad sync word
    jobs[5].stations[1].frames = jobs[5].stations[1].frames[:-2].contiguous()   # cut short
    # a second job over job 1's recordings (the same tensors), a later stretch of time
    jobs.append(dataclasses.replace(jobs[1], n_frames=100, sub_start=jobs[1].sub_start + 20 * 256))
    precs.append(xc.XC_FP32)
    # handed to single-job runs
    jobs.append(configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=16384, C=1,
                                  n_frames=3, seed=520))
    precs.append(xc.XC_FP32)
    jobs.append(configs.small_job(n_stations=4, n_subbands=2, n_pols=1, n_chan=256, C=2,
                                  n_frames=60, seed=521))
    precs.append(xc.XC_FP16_MFMA)
    rc = configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=1024, C=1, n_frames=20,
                           seed=522)
    rc = dataclasses.replace(rc, stations=[dataclasses.replace(rc.stations[0], rate_correct=True),
                                           rc.stations[1]])
    jobs.append(rc)
    precs.append(xc.XC_FP32)
    for j in jobs:
        xc.job_to_device(j)
    return jobs, precs


@pytest.mark.parametrize("fpb", [0, 64])
def test_fused_executor_corner_cases(xc, corr, fpb):
    """The fused executor over the corner-case mix, in one block per job
    (fpb = 0) and in 64-frame blocks (jobs of two to four blocks run in rounds,
    job 0's five blocks make it a single job), with and without graph capture:
    identical to each job run alone at the same block size; the FP32 jobs
    within tolerance of the oracle."""
    jobs, precs = _fused_mix(xc)
    try:
        corr.set_tuning(frames_per_block=fpb)
        refs = [tuple(x.clone() for x in corr.correlate(j, precision=p))
                for j, p in zip(jobs, precs)]
        for graph in (False, True):
            ws = corr.batch_workspace(jobs, n_lanes=3, precision=precs)
            outs = [corr.alloc_output(j) for j in jobs]
            for rep in range(2 if graph else 1):
                for v, w in outs:
                    v.zero_()
                    w.zero_()
                corr.correlate_batch(jobs, n_lanes=3, graph=graph, precision=precs, outs=outs,
                                     workspace=ws)
                torch.cuda.synchronize()
                for k, ((v, w), (rv, rw)) in enumerate(zip(outs, refs)):
                    assert torch.equal(v, rv) and torch.equal(w, rw), (fpb, graph, rep, k)
    finally:
        corr.set_tuning(frames_per_block=0)
    if fpb == 64:
        for k in (1, 4, 5, 9):
            V, W = fx.correlate(jobs[k], threads=8)
            assert np.array_equal(refs[k][1].cpu().numpy(), W.astype(np.float32)), k
            assert rel_l2(refs[k][0].cpu().numpy(), V) < 1e-5, k


def test_long_job_keeps_default_block(xc, corr):
    """A job that the batch's 1 GiB bound on staged spectra would cut into more
    than four blocks keeps the library's default block (here the whole job) and
    runs alone on the first lane: with both executors, with and without graph
    capture, every job of the batch equals the job run alone with the library
    defaults, bit for bit (the long job's FP64 slot sums would differ in order
    at the bounded block size)."""
    big = configs.small_job("cuda", n_stations=5, n_subbands=8, n_pols=2, n_chan=1024, C=16,
                            n_frames=6600, seed=31, realistic=True)
    per_frame = 8 * 10 * 1024 * 8                        # FP32 spectra per frame
    assert -(-big.n_frames // ((1 << 30) // per_frame)) == 5
    jobs = [big] + _jobs(xc)[:5]
    for j in jobs[1:]:
        xc.job_to_device(j)
    refs = [tuple(x.clone() for x in corr.correlate(j)) for j in jobs]
    for lanes_only in (False, True):
        ws = corr.batch_workspace(jobs, n_lanes=3, lanes_only=lanes_only)
        for graph in (False, True):
            outs = [corr.alloc_output(j) for j in jobs]
            corr.correlate_batch(jobs, n_lanes=3, graph=graph, lanes_only=lanes_only, outs=outs,
                                 workspace=ws)
            torch.cuda.synchronize()
            for k, ((v, w), (rv, rw)) in enumerate(zip(outs, refs)):
                assert torch.equal(v, rv) and torch.equal(w, rw), (lanes_only, graph, k)
        del ws


def test_fused_batch_with_tuned_matrix_ring(xc, corr):
    """Jobs tuned to the matrix-core ring X stage (the fused executor's own X
    kernel, whose sums equal the vector ring's) stay fusable: with and without
    graph capture the batch equals each job run alone with that tuning."""
    jobs = _jobs(xc)[:6]
    for j in jobs:
        xc.job_to_device(j)
    try:
        corr.set_tuning(xmac_frames_per_stage=5)
        refs = [tuple(x.clone() for x in corr.correlate(j)) for j in jobs]
        ws = corr.batch_workspace(jobs, n_lanes=2)
        for graph in (False, True):
            outs = [corr.alloc_output(j) for j in jobs]
            corr.correlate_batch(jobs, n_lanes=2, graph=graph, outs=outs, workspace=ws)
            torch.cuda.synchronize()
            for k, ((v, w), (rv, rw)) in enumerate(zip(outs, refs)):
                assert torch.equal(v, rv) and torch.equal(w, rw), (graph, k)
    finally:
        corr.set_tuning(xmac_frames_per_stage=0)


def test_batch_against_oracle(xc, corr, batch):
    jobs, refs = batch
    for i in (0, 5, 11):
        V, W = fx.correlate(jobs[i], threads=8)
        v, w = refs[i]
        assert np.array_equal(w.cpu().numpy(), W.astype(np.float32))
        assert rel_l2(v.cpu().numpy(), V) < 1e-5


def test_graph_capture_and_replay(xc, corr, batch):
    jobs, refs = batch
    ws = corr.batch_workspace(jobs, n_lanes=4)
    outs = [corr.alloc_output(j) for j in jobs]
    for rep in range(3):
        for v, w in outs:
            v.zero_()
            w.zero_()
        torch.cuda.synchronize()
        corr.correlate_batch(jobs, n_lanes=4, graph=True, outs=outs, workspace=ws)
        torch.cuda.synchronize()
        for (v, w), (rv, rw) in zip(outs, refs):
            assert torch.equal(v, rv) and torch.equal(w, rw), rep


def test_batch_mixed_precision(xc, corr):
    jobs = [configs.small_job(n_stations=4, n_subbands=2, n_pols=1, n_chan=256, C=2, n_frames=80,
                              seed=7 + i) for i in range(3)]
    for j in jobs:
        xc.job_to_device(j)
    precs = [xc.XC_FP32, xc.XC_FP16_MFMA, xc.XC_FP32]
    refs = [corr.correlate(j, precision=p) for j, p in zip(jobs, precs)]
    outs = corr.correlate_batch(jobs, n_lanes=2, precision=precs)
    torch.cuda.synchronize()
    for (v, w), (rv, rw) in zip(outs, refs):
        assert torch.equal(v, rv) and torch.equal(w, rw)


def test_batch_rejects_bad_job(xc, corr, batch):
    jobs, _ = batch
    bad = configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=10)
    xc.job_to_device(bad)
    bad.stations[0].poly_span = (0.0, 1.0)
    with pytest.raises(xc.XcError) as e:
        corr.correlate_batch(jobs[:2] + [bad], n_lanes=2)
    assert e.value.code == xc.XC_E_RANGE and "job 2" in str(e.value)


def test_autotune_picks_a_candidate_and_stays_correct(xc, corr):
    job = configs.small_job(n_stations=5, n_subbands=2, n_pols=2, n_chan=512, C=4, n_frames=900)
    V, W = fx.correlate(job, threads=8)
    xc.job_to_device(job)
    best = corr.autotune(job)
    assert best["frames_per_block"] == 0           # the library default block (it fits)
    assert best["xmac_frames_per_stage"] in (0, 1, 2, 3, 4, 5, 8)
    vis, w = corr.correlate(job)           # uses the tuned shape
    assert rel_l2(vis.cpu().numpy(), V) < 1e-5
