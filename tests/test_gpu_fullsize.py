"""GPU parity at full configuration sizes, in the launch configuration bench.py times.

The oracle recomputes sampled outputs over the whole sub-integration (all
frames): C1 completely (it fits), C2 and C4 for sampled subbands and inputs.
"""
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


def _host_copy(job):
    """A host-side view of the job for the oracle (recordings copied from the GPU)."""
    import copy
    h = copy.copy(job)
    h.stations = [copy.copy(st) for st in job.stations]
    for st in h.stations:
        st.frames = st.frames.cpu()
    return h


@pytest.mark.timeout(300)
def test_c1_full(xc, corr):
    print("\nC1: generating 2 x 16e6 samples (exact physics)", flush=True)
    job = configs.c1_job(device="cuda")
    xc.job_to_device(job)
    vis, w = corr.correlate(job)
    torch.cuda.synchronize()
    print("C1: oracle on all 31250 frames", flush=True)
    V, W = fx.correlate(_host_copy(job), threads=16)
    assert np.array_equal(w.cpu().numpy(), W.astype(np.float32))
    err = rel_l2(vis.cpu().numpy(), V)
    print(f"C1 full: max rel L2 per baseline {err:.2e}", flush=True)
    assert err < TOL
    # the GPU result shows the injected delay at the oracle's lag
    v = vis.cpu().numpy()[0, 1].astype(np.complex128)
    m = np.arange(130, 145, 1.0 / 16)
    L = np.exp(-2j * np.pi * np.outer(m, np.arange(256)) / 512) @ v
    assert abs(m[np.argmax(np.abs(L))] - 137.25) <= 0.05


@pytest.mark.timeout(300)
def test_c2_full_sampled(xc, corr):
    print("\nC2: generating 10 stations x 16 streams x 4 s on the GPU", flush=True)
    job = configs.c2_job(device="cuda", realistic=True)
    vis, w = corr.correlate(job)                        # bench launch configuration
    torch.cuda.synchronize()
    v, ww = vis.cpu().numpy(), w.cpu().numpy()
    M = job.M
    # subband 3: the space station's two pols and station 6 pol 1; subband 6:
    # stations 2 and 9, both pols (2 of the 8 subbands, 16 of their 420 products)
    for sb, inputs in ((3, [0, 1, 13]), (6, [4, 5, 18, 19])):
        host = _host_copy(job)
        used = {i // 2 for i in inputs}
        for s_, st in enumerate(host.stations):
            if s_ not in used:
                st.frames = st.frames[:1]               # unused stations: no host copy needed
        print(f"C2: oracle on subband {sb}, inputs {inputs}, all 62500 frames", flush=True)
        V, W = fx.correlate(host, subbands=[sb], inputs=inputs, threads=16)
        for a in inputs:
            for b in inputs:
                if a > b:
                    continue
                bl = fx.baseline_index(a, b, M)
                assert ww[sb, bl] == W[sb, bl] == job.n_frames
                e = rel_l2(v[sb, bl], V[sb, bl])
                print(f"C2 full, subband {sb}, ({a},{b}): rel L2 {e:.2e}", flush=True)
                assert e < TOL


@pytest.mark.timeout(300)
def test_c4_full_sampled_all_precisions(xc, corr):
    print("\nC4: generating 32 stations x 4 streams x 1 s on the GPU", flush=True)
    job = configs.c4_job(device="cuda")
    host = _host_copy(job)
    sb, inputs = 0, [0, 17, 31]
    V, W = fx.correlate(host, subbands=[sb], inputs=inputs, threads=16)
    M = job.M
    for prec, u in (("fp32", None), ("fp16", 2.0 ** -11), ("fp8", 2.0 ** -4)):
        vis, w = corr.correlate(job, precision=xc.PRECISIONS[prec])
        torch.cuda.synchronize()
        v = vis.cpu().numpy()
        for a in inputs:
            for b in inputs:
                if a > b:
                    continue
                bl = fx.baseline_index(a, b, M)
                if u is None:
                    assert rel_l2(v[sb, bl], V[sb, bl]) < TOL
                else:
                    A = V[sb, fx.baseline_index(a, a, M)].real
                    B = V[sb, fx.baseline_index(b, b, M)].real
                    d = np.max(np.abs(v[sb, bl] - V[sb, bl]) / np.sqrt(A * B))
                    print(f"C4 {prec} ({a},{b}): max |dV|/sqrt(AiAj) {d:.2e}", flush=True)
                    assert d <= 1.1 * (2 * u + u * u)
