"""GPU parity: feed-angle correction (xc_feed_correct) against oracle/feed.py."""
import numpy as np
import pytest
import torch

from oracle import feed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xc():
    from paper_1502_06894_amd import xcorr
    return xcorr


@pytest.fixture(scope="module")
def corr(xc):
    return xc.Correlator(0)


@pytest.mark.parametrize("kind", [feed.CIRCULAR, feed.LINEAR])
@pytest.mark.parametrize("S,T,n_sb,n_chan", [(5, 3, 2, 100), (1, 1, 1, 1), (10, 2, 8, 1024),
                                             (3, 2, 1, 1537), (16, 1, 2, 2050), (2, 1, 3, 4096)])
def test_feed_parity(xc, corr, kind, S, T, n_sb, n_chan):
    rng = np.random.default_rng(S * 100 + kind)
    M = 2 * S
    nbl = M * (M + 1) // 2
    V = (rng.normal(size=(T, n_sb, nbl, n_chan)) + 1j * rng.normal(size=(T, n_sb, nbl, n_chan)))
    V = V.astype(np.complex64)
    ang = rng.uniform(-np.pi, np.pi, size=(T, S))
    want = feed.correct(V.astype(np.complex128), ang, kind)
    vis = torch.from_numpy(V).cuda()
    corr.feed_correct(vis, torch.from_numpy(ang).cuda(), kind)
    got = vis.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 2e-6 * np.max(np.abs(want))


@pytest.mark.parametrize("kind", [feed.CIRCULAR, feed.LINEAR])
def test_feed_unaligned_buffer(xc, corr, kind):
    """A buffer that starts 8 bytes past a 16-byte boundary takes the one-channel path."""
    rng = np.random.default_rng(31 + kind)
    S, T, n_sb, n_chan = 4, 2, 2, 512
    M = 2 * S
    nbl = M * (M + 1) // 2
    V = (rng.normal(size=(T, n_sb, nbl, n_chan)) + 1j * rng.normal(size=(T, n_sb, nbl, n_chan)))
    ang = rng.uniform(-np.pi, np.pi, size=(T, S))
    want = feed.correct(V, ang, kind)
    flat = torch.zeros(V.size + 1, dtype=torch.complex64, device="cuda")
    vis = flat[1:].view(T, n_sb, nbl, n_chan)
    assert vis.data_ptr() % 16 == 8
    vis.copy_(torch.from_numpy(V.astype(np.complex64)))
    corr.feed_correct(vis, torch.from_numpy(ang).cuda(), kind)
    got = vis.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 2e-6 * np.max(np.abs(want))
    assert flat[0].item() == 0


def test_feed_errors(xc, corr):
    vis = torch.zeros((1, 1, 3, 4), dtype=torch.complex64, device="cuda")
    with pytest.raises(xc.XcError) as e:
        corr.feed_correct(vis, torch.zeros((1, 1), dtype=torch.float64, device="cuda"), 7)
    assert e.value.code == xc.XC_E_INVAL
    with pytest.raises(xc.XcError):                      # 3 products need S = 1, not 2
        corr.feed_correct(vis, torch.zeros((1, 2), dtype=torch.float64, device="cuda"), 0)
    with pytest.raises(xc.XcError):                      # one angle row per sub-integration
        corr.feed_correct(vis, torch.zeros((2, 1), dtype=torch.float64, device="cuda"), 0)
