"""GPU: the continuous-batching server.

Each result must be bit-identical alone (plain path) and in the mix (served
concurrently with other requests, arriving while others run); admission by
HBM footprint, rejection of oversized requests, cancel and time-out.
"""
import time

import numpy as np
import pytest
import torch

from synth import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xc():
    from paper_1502_06894_amd import xcorr
    return xcorr


@pytest.fixture(scope="module")
def corr(xc):
    return xc.Correlator(0)


@pytest.fixture(scope="module")
def jobs_and_refs(xc, corr):
    rng = np.random.default_rng(77)
    jobs, refs = [], []
    for i in range(10):
        j = configs.small_job(n_stations=int(rng.integers(2, 8)), n_subbands=int(rng.integers(1, 4)),
                              n_pols=1, n_chan=int(2 ** rng.integers(7, 11)), C=4,
                              n_frames=int(rng.integers(20, 400)), seed=300 + i)
        xc.job_to_device(j)
        v, w = corr.correlate(j)
        jobs.append(j)
        refs.append((v.clone(), w.clone()))
    torch.cuda.synchronize()
    return jobs, refs


def test_alone_equals_in_the_mix(xc, jobs_and_refs):
    jobs, refs = jobs_and_refs
    srv = xc.Server(0, hbm_budget_bytes=4 << 30, max_slots=4)
    try:
        tickets = []
        for k, j in enumerate(jobs):
            tickets.append(srv.submit(j))
            if k % 3 == 2:
                time.sleep(0.002)          # later requests arrive while earlier ones run
        for (t, (v, w)), (rv, rw) in zip(tickets, refs):
            assert srv.wait(t, 60000) == xc.XC_OK
            assert torch.equal(v, rv) and torch.equal(w, rw)
        st = srv.stats()
        assert st["completed"] == len(jobs) and st["failed"] == 0
        assert st["p99_ms"] >= st["p50_ms"] > 0 and st["station_samples_per_s"] > 0
    finally:
        srv.close()


def test_admission_by_footprint(xc, corr, jobs_and_refs):
    jobs, refs = jobs_and_refs
    fps = [corr.workspace_bytes(j) for j in jobs]
    srv = xc.Server(0, hbm_budget_bytes=max(fps) + (1 << 20), max_slots=4)   # ~one at a time
    try:
        tickets = [srv.submit(j) for j in jobs]
        for (t, (v, w)), (rv, rw) in zip(tickets, refs):
            assert srv.wait(t, 60000) == xc.XC_OK
            assert torch.equal(v, rv) and torch.equal(w, rw)
        with pytest.raises(xc.XcError) as e:      # can never fit
            small = xc.Server(0, hbm_budget_bytes=1 << 20, max_slots=1)
            try:
                small.submit(jobs[0])
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
