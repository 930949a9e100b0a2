"""GPU: the continuous-batching server.

Each result must be bit-identical alone (plain path) and in the mix (served
concurrently with other requests, arriving while others run); the plain-path
results themselves are checked against the FP64 oracle, so the served ones
are too.  Also: admission by HBM footprint, rejection of oversized requests,
cancel and time-out, and that a reported ticket is retired.
"""
import time

import numpy as np
import pytest
import torch

from oracle import fx
from synth import configs
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5
U16 = 2.0 ** -11          # FP16 unit roundoff (MFMA X stage)


@pytest.fixture(scope="module")
def xc():
    from paper_1502_06894_amd import xcorr
    return xcorr


@pytest.fixture(scope="module")
def corr(xc):
    return xc.Correlator(0)


def _mix():
    """Ten single-pol jobs of random shape, a dual-pol job, a 16384-channel job
    (N = 32768: the folded FP32 F stage) and an FP16 (MFMA) job."""
    rng = np.random.default_rng(77)
    jobs = []
    for i in range(10):
        jobs.append((configs.small_job(n_stations=int(rng.integers(2, 8)),
                                       n_subbands=int(rng.integers(1, 4)), n_pols=1,
                                       n_chan=int(2 ** rng.integers(7, 11)), C=4,
                                       n_frames=int(rng.integers(20, 400)), seed=300 + i), 0))
    jobs.append((configs.small_job(n_stations=4, n_subbands=3, n_pols=2, n_chan=512, C=8,
                                   n_frames=150, seed=320), 0))
    jobs.append((configs.small_job(n_stations=3, n_subbands=1, n_pols=2, n_chan=16384, C=2,
                                   n_frames=5, seed=321), 0))
    jobs.append((configs.small_job(n_stations=5, n_subbands=2, n_pols=1, n_chan=1024, C=2,
                                   n_frames=90, seed=322), 1))
    return jobs


@pytest.fixture(scope="module")
def jobs_and_refs(xc, corr):
    jobs, refs = [], []
    for j, prec in _mix():
        xc.job_to_device(j)
        v, w = corr.correlate(j, precision=prec)
        jobs.append((j, prec))
        refs.append((v.clone(), w.clone()))
    torch.cuda.synchronize()
    return jobs, refs


def test_plain_results_match_the_oracle(xc, jobs_and_refs):
    """The references the served results are compared with bit for bit are
    themselves within tolerance of the FP64 oracle (FP32 jobs: relative L2
    per baseline; the FP16 job: the per-element rounding bound
    (2u + u^2) sqrt(A_i A_j) with 10 % slack)."""
    jobs, refs = jobs_and_refs
    for (job, prec), (v, w) in zip(jobs, refs):
        V, W = fx.correlate(job, threads=8)
        vis, w = v.cpu().numpy(), w.cpu().numpy()
        assert np.array_equal(w, W.astype(np.float32))
        if prec == 0:
            for sb in range(job.n_subbands):
                for bl in range(job.n_baselines):
                    assert rel_l2(vis[sb, bl], V[sb, bl]) < TOL, (job.n_chan, sb, bl)
        else:
            M = job.M
            for sb in range(job.n_subbands):
                for i in range(M):
                    for j in range(i, M):
                        bl = fx.baseline_index(i, j, M)
                        A = np.sqrt(V[sb, fx.baseline_index(i, i, M)].real *
                                    V[sb, fx.baseline_index(j, j, M)].real)
                        d = np.abs(vis[sb, bl] - V[sb, bl]) / A
                        assert d.max() <= 1.1 * (2 * U16 + U16 * U16), (sb, i, j)


def test_alone_equals_in_the_mix(xc, jobs_and_refs):
    jobs, refs = jobs_and_refs
    srv = xc.Server(0, hbm_budget_bytes=8 << 30, max_slots=4)
    try:
        tickets = []
        for k, (j, prec) in enumerate(jobs):
            tickets.append(srv.submit(j, precision=prec))
            if k % 3 == 2:
                time.sleep(0.002)          # later requests arrive while earlier ones run
        for (t, (v, w)), (rv, rw) in zip(tickets, refs):
            assert srv.wait(t, 60000) == xc.XC_OK
            assert torch.equal(v, rv) and torch.equal(w, rw)
        st = srv.stats()
        assert st["completed"] == len(jobs) and st["failed"] == 0
        assert st["p99_ms"] >= st["p50_ms"] > 0 and st["station_samples_per_s"] > 0
        # a ticket whose result was reported is retired
        assert srv.wait(tickets[0][0], 0) == xc.XC_E_INVAL
        assert srv.poll(tickets[1][0])[1] == xc.XC_E_INVAL
    finally:
        srv.close()


def test_admission_by_footprint(xc, corr, jobs_and_refs):
    jobs, refs = jobs_and_refs
    fps = [corr.workspace_bytes(j, precision=p) for j, p in jobs]
    srv = xc.Server(0, hbm_budget_bytes=max(fps) + (1 << 20), max_slots=4)   # ~one at a time
    try:
        tickets = [srv.submit(j, precision=p) for j, p in jobs]
        for (t, (v, w)), (rv, rw) in zip(tickets, refs):
            assert srv.wait(t, 60000) == xc.XC_OK
            assert torch.equal(v, rv) and torch.equal(w, rw)
        with pytest.raises(xc.XcError) as e:      # can never fit
            small = xc.Server(0, hbm_budget_bytes=1 << 20, max_slots=1)
            try:
                small.submit(jobs[0][0])
            finally:
                small.close()
        assert e.value.code == xc.XC_E_NOMEM
    finally:
        srv.close()


def test_cancel_and_timeout(xc):
    big = configs.small_job(n_stations=10, n_subbands=4, n_pols=2, n_chan=1024, C=8, n_frames=3000,
                            seed=5)
    small = configs.small_job(n_stations=2, n_subbands=1, n_pols=1, n_chan=256, C=1, n_frames=50,
                              seed=6)
    xc.job_to_device(big)
    xc.job_to_device(small)
    srv = xc.Server(0, hbm_budget_bytes=16 << 30, max_slots=1)
    try:
        t1, _ = srv.submit(big)
        t2, _ = srv.submit(small)
        assert srv.wait(t1, 0) == xc.XC_E_TIMEOUT
        assert srv.cancel(t2) == xc.XC_OK
        assert srv.wait(t2, 60000) == xc.XC_E_CANCELLED
        assert srv.wait(t1, 60000) == xc.XC_OK
        assert srv.cancel(t1) == xc.XC_E_INVAL           # already finished
        st = srv.stats()
        assert st["cancelled"] == 1 and st["completed"] == 1
    finally:
        srv.close()
