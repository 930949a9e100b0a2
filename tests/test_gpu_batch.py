"""GPU: batches (lanes, hipGraph capture/replay) and the autotuner.

A batch must reproduce each job's stand-alone result bit for bit (the same
kernels and summation order run, only concurrently), for any lane count and
on graph replay; a few jobs are also checked against the FP64 oracle.
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
    for lanes in (1, 3, 8):
        outs = corr.correlate_batch(jobs, n_lanes=lanes)
        torch.cuda.synchronize()
        for (v, w), (rv, rw) in zip(outs, refs):
            assert torch.equal(v, rv) and torch.equal(w, rw), lanes


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
    assert best["frames_per_block"] in (512, 1024, 2048)
    assert best["xmac_frames_per_stage"] in (1, 2, 4, 8)
    vis, w = corr.correlate(job)           # uses the tuned shape
    assert rel_l2(vis.cpu().numpy(), V) < 1e-5
