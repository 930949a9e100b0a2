"""GPU: the allocation-free entry point (xc_correlate_subint_noalloc) against
xc_correlate_subint, through the C ABI.

At the same frames per block both run the same kernels in the same order, so
the results must be identical bit for bit; with the block size left to the
library the allocation-free call picks a block that fits its fixed scratch,
and its results stay within the FP32 tolerance of the workspace call's.  Two
calls in a row (the second on a smaller job) check that what the first left
in the shared scratch does not leak into the second.
"""
import numpy as np
import pytest
import torch

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


def test_noalloc_matches_workspace_call(xc, corr):
    big = configs.small_job(n_stations=6, n_subbands=2, n_pols=2, n_chan=1024, C=4, n_frames=300,
                            seed=61)
    small = configs.small_job(n_stations=3, n_subbands=1, n_pols=1, n_chan=256, C=2, n_frames=50,
                              seed=62)
    for j in (big, small):
        xc.job_to_device(j)
    for job, fpb in ((big, 64), (small, 16)):
        ref_v, ref_w = corr.correlate(job, frames_per_block=fpb)
        v, w = corr.correlate_noalloc(job, frames_per_block=fpb)
        torch.cuda.synchronize()
        assert torch.equal(v, ref_v) and torch.equal(w, ref_w), fpb
    for job in (big, small):
        ref_v, ref_w = corr.correlate(job)
        v, w = corr.correlate_noalloc(job)
        torch.cuda.synchronize()
        assert torch.equal(w, ref_w)
        assert rel_l2(v.cpu().numpy(), ref_v.cpu().numpy()) < TOL


def test_noalloc_picks_a_block_that_fits(xc, corr):
    """A job whose default block would not fit the scratch: the call picks a
    smaller block (results within tolerance of the workspace call); a fixed
    block size that does not fit is refused with XC_E_NOMEM."""
    job = configs.c2_job(n_frames=300, n_subbands=8, n_stations=10)
    xc.job_to_device(job)
    cap = xc.load_library().xc_noalloc_scratch_bytes()
    assert corr.workspace_bytes(job) > cap
    ref_v, ref_w = corr.correlate(job)
    v, w = corr.correlate_noalloc(job)
    torch.cuda.synchronize()
    assert torch.equal(w, ref_w)
    assert rel_l2(v.cpu().numpy(), ref_v.cpu().numpy()) < TOL
    with pytest.raises(xc.XcError) as e:
        corr.correlate_noalloc(job, frames_per_block=300)
    assert e.value.code == xc.XC_E_NOMEM
