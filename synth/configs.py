"""The five workload configurations as concrete, seeded parameters.

  C1  2 stations (ground + space), 1 x 16 MHz, single pol, 256 channels,
      0.5 s (16 000 000 samples), exact-physics generator, residual delay of
      137.25 samples on the space station, correlation coefficient 0.05.
  C2  10 stations (1 space + 9 ground), 8 x 16 MHz, dual pol (16 recorded
      streams), 1024 channels, 4 s.
  C3  64 uneven batch jobs (see batch_jobs).
  C4  32 stations, 4 x 32 MHz (64 Msps, 4 streams), single pol, 4096 channels, 1 s.
  C5  Poisson request trace (see serve_trace).

The observing band starts at 4.82 GHz (the 4.9 GHz band of the paper's first
RadioAstron image); subband sb's lower edge is 4.82 GHz + sb * bandwidth.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from . import physics, shape
from .job import Job

MASTER_SEED = 1502068940
LO0_HZ = 4.82e9
FS_16MHZ = 32e6

# delay polynomials (seconds, ascending powers of t = seconds since the epoch)
GROUND_C1 = [-0.0123, 2.1e-6, -1e-11, 0.0, 0.0, 0.0]
SPACE_C1 = [0.40, 1.0e-5, 3e-10, -2e-13, 1e-16, -4e-20]
SUB_START_S = 37.0
C1_RESIDUAL_SAMPLES = 137.25


def cfg_seed(c: int) -> int:
    return MASTER_SEED + c


def ground_poly(rng: np.random.Generator) -> List[float]:
    return [float(rng.uniform(-0.02, 0.02)), float(rng.uniform(-3e-6, 3e-6)),
            float(rng.uniform(-1e-11, 1e-11)), 0.0, 0.0, 0.0]


def c1_job(n_frames: int = 31250, seed: int | None = None, device="cpu") -> Job:
    """C1: exact-physics two-station job (torch work on `device`)."""
    fs, N = FS_16MHZ, 512
    return physics.two_station_job(
        fs=fs, N=N, n_frames=n_frames, sub_start=int(SUB_START_S * fs),
        model_polys=[GROUND_C1, SPACE_C1],
        residual_delay_s=[0.0, C1_RESIDUAL_SAMPLES / fs],
        lo_hz=LO0_HZ, rho=0.05, seed=cfg_seed(1) if seed is None else seed, name="C1",
        device=device)


def c2_job(device="cpu", n_frames: int = 62500, n_subbands: int = 8, n_stations: int = 10,
           realistic: bool = True, seed: int | None = None, n_chan: int = 1024) -> Job:
    """C2: 10 stations, 8 x 16 MHz dual pol, 1024 channels, 4 s (62 500 frames).

    realistic=True: space polynomial as C1 plus random ground polynomials and
    fringe phase nu*tau (used for timing).  realistic=False: constant
    polynomials matched to the sky shifts and zero phase (physically consistent).
    """
    seed = cfg_seed(2) if seed is None else seed
    rng = np.random.default_rng(seed)
    fs = FS_16MHZ
    shifts = [int(v) for v in rng.integers(-2000, 2001, size=n_stations)]
    if realistic:
        polys = [SPACE_C1] + [ground_poly(rng) for _ in range(n_stations - 1)]
    else:
        polys = [[s / fs, 0.0, 0.0, 0.0, 0.0, 0.0] for s in shifts]
    lo = [LO0_HZ + sb * 16e6 for sb in range(n_subbands)]
    return shape.build_job(n_stations=n_stations, n_subbands=n_subbands, n_pols=2,
                           n_chan=n_chan, C=16, fs=fs, lo_hz=lo,
                           sub_start=int(SUB_START_S * fs), n_frames=n_frames,
                           delay_polys=polys, shifts=shifts, phase_zero=not realistic,
                           seed=seed, device=device, name="C2")


def c4_job(device="cpu", n_frames: int = 7812, n_stations: int = 32, n_subbands: int = 4,
           realistic: bool = False, seed: int | None = None, n_chan: int = 4096) -> Job:
    """C4: 32 stations, 4 x 32 MHz (64 Msps, C = 4), single pol, 4096 channels, 1 s."""
    seed = cfg_seed(4) if seed is None else seed
    rng = np.random.default_rng(seed)
    fs = 64e6
    shifts = [int(v) for v in rng.integers(-2000, 2001, size=n_stations)]
    if realistic:
        polys = [SPACE_C1] + [ground_poly(rng) for _ in range(n_stations - 1)]
    else:
        polys = [[s / fs, 0.0, 0.0, 0.0, 0.0, 0.0] for s in shifts]
    lo = [LO0_HZ + sb * 32e6 for sb in range(n_subbands)]
    return shape.build_job(n_stations=n_stations, n_subbands=n_subbands, n_pols=1,
                           n_chan=n_chan, C=4, fs=fs, lo_hz=lo,
                           sub_start=int(SUB_START_S * fs), n_frames=n_frames,
                           delay_polys=polys, shifts=shifts, phase_zero=not realistic,
                           seed=seed, device=device, name="C4")


def small_job(device="cpu", *, n_stations=3, n_subbands=2, n_pols=2, n_chan=256, C=4,
              n_frames=40, fs=FS_16MHZ, realistic=True, seed=7, stream_map=None,
              sub_start_s=SUB_START_S, phase_zero=None) -> Job:
    """Small mixed job for tests: space station 0, ground stations after it."""
    rng = np.random.default_rng(seed)
    shifts = [int(v) for v in rng.integers(-200, 201, size=n_stations)]
    if realistic:
        polys = [SPACE_C1] + [ground_poly(rng) for _ in range(n_stations - 1)]
    else:
        polys = [[s / fs, 0.0, 0.0, 0.0, 0.0, 0.0] for s in shifts]
    bw = fs / 2
    lo = [LO0_HZ + sb * bw for sb in range(n_subbands)]
    pz = (not realistic) if phase_zero is None else phase_zero
    return shape.build_job(n_stations=n_stations, n_subbands=n_subbands, n_pols=n_pols,
                           n_chan=n_chan, C=C, fs=fs, lo_hz=lo,
                           sub_start=int(round(sub_start_s * fs)), n_frames=n_frames,
                           delay_polys=polys, shifts=shifts, phase_zero=pz, seed=seed,
                           device=device, margin=1024, stream_map=stream_map, name="small")


# ---------------------------------------------------------------- C3 / C5: jobs over a pool

POOL_STATIONS = 20
POOL_STREAMS = 16
POOL_SECONDS = 4.5
POOL_T0_S = 37.0


def pool_recordings(device="cpu", seed: int | None = None, seconds: float = POOL_SECONDS,
                    n_stations: int = POOL_STATIONS):
    """Device-resident recordings shared by batch and serving jobs: n_stations x 16
    streams x `seconds` at 32 Msps (11.5 GB for the full pool), ground-station-like
    delays; returns (stations' frames, first_sample, delay polynomials)."""
    from . import format as fmt
    from .shape import _Sky, make_station_frames
    seed = cfg_seed(3) if seed is None else seed
    rng = np.random.default_rng(seed)
    fs, C = FS_16MHZ, POOL_STREAMS
    polys = [[float(rng.uniform(-0.02, 0.02)), float(rng.uniform(-3e-6, 3e-6)), 0.0, 0.0, 0.0, 0.0]
             for _ in range(n_stations)]
    spf = fmt.samples_per_frame(C)
    first = int(POOL_T0_S * fs)
    n_m5b = -(-int(seconds * fs) // spf)
    sky = _Sky(C, seed, device)
    frames = [make_station_frames(C=C, fs=fs, first_sample=first, n_m5b=n_m5b,
                                  shift=int(round(polys[s][0] * fs)), station_id=s, sky=sky,
                                  seed=seed, rho=0.05, device=device) for s in range(n_stations)]
    return frames, first, polys


def pool_job(frames, first, polys, *, stations, n_subbands, n_chan, seconds, start_s, streams,
             name="") -> Job:
    """A single-pol job over pool stations `stations`, subbands on `streams`."""
    from .job import Station
    fs = FS_16MHZ
    N = 2 * n_chan
    n_frames = max(1, int(seconds * fs) // N)
    sts = [Station(frames=frames[s], first_sample=first,
                   delay_poly=np.asarray(polys[s], dtype=np.float64), station_id=s)
           for s in stations]
    return Job(n_stations=len(stations), n_subbands=n_subbands, n_pols=1, n_chan=n_chan,
               n_streams=POOL_STREAMS, stream_map=list(streams), fs_hz=fs,
               lo_hz=[LO0_HZ + s * 16e6 for s in streams],
               sub_start=int(round((POOL_T0_S + start_s) * fs)), n_frames=n_frames,
               stations=sts, name=name)


def _random_pool_job(rng, pool, *, s_range, sb_range, log2_chan, len_range, pool_seconds):
    frames, first, polys = pool
    S = int(rng.integers(s_range[0], s_range[1] + 1))
    nsb = int(rng.integers(sb_range[0], sb_range[1] + 1))
    n_chan = int(2 ** rng.integers(log2_chan[0], log2_chan[1] + 1))
    length = float(rng.uniform(*len_range))
    length = min(length, pool_seconds - 0.1)
    start = float(rng.uniform(0.05, pool_seconds - 0.05 - length))
    stations = sorted(rng.choice(len(frames), size=min(S, len(frames)), replace=False).tolist())
    streams = sorted(rng.choice(POOL_STREAMS, size=nsb, replace=False).tolist())
    return pool_job(frames, first, polys, stations=stations, n_subbands=nsb, n_chan=n_chan,
                    seconds=length, start_s=start, streams=streams)


def batch_jobs(pool, n_jobs: int = 64, seed: int | None = None,
               pool_seconds: float = POOL_SECONDS):
    """C3: uneven sub-integrations: stations U{2..20}, subbands U{1..16},
    channels 2^U{7..13}, lengths U[0.1, 4] s, single pol, 32 Msps."""
    rng = np.random.default_rng(cfg_seed(3) + 1 if seed is None else seed)
    return [_random_pool_job(rng, pool, s_range=(2, 20), sb_range=(1, 16), log2_chan=(7, 13),
                             len_range=(0.1, 4.0), pool_seconds=pool_seconds)
            for _ in range(n_jobs)]


def short_batch_jobs(pool, n_jobs: int = 256, seed: int | None = None,
                     pool_seconds: float = POOL_SECONDS):
    """Many short sub-integrations, each too small to fill the GPU alone:
    stations U{2..6}, subbands U{1..4}, channels 2^U{7..10}, lengths
    U[0.01, 0.1] s, single pol, 32 Msps."""
    rng = np.random.default_rng(cfg_seed(3) + 2 if seed is None else seed)
    return [_random_pool_job(rng, pool, s_range=(2, 6), sb_range=(1, 4), log2_chan=(7, 10),
                             len_range=(0.01, 0.1), pool_seconds=pool_seconds)
            for _ in range(n_jobs)]


def serve_trace(pool, n_requests: int = 2000, rate_hz: float = 200.0, seed: int | None = None,
                pool_seconds: float = POOL_SECONDS, max_log2_chan: int = 14):
    """C5: Poisson arrivals (seeded exponential gaps) of requests with stations
    U{3..20}, subbands U{1..16}, channels 2^U{8..14}, lengths U[0.1, 4] s.
    Returns [(arrival_s, job)]."""
    rng = np.random.default_rng(cfg_seed(5) if seed is None else seed)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        out.append((t, _random_pool_job(rng, pool, s_range=(3, 20), sb_range=(1, 16),
                                        log2_chan=(8, max_log2_chan), len_range=(0.1, 4.0),
                                        pool_seconds=pool_seconds)))
    return out
