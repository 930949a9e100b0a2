"""Test helpers: jobs built from explicit 2-bit codes (no correlator arithmetic)."""
from __future__ import annotations

import numpy as np
import torch

from synth import format as fmt
from synth.job import Job, Station


def station_from_codes(codes: np.ndarray, C: int, first_sample: int, delay_poly,
                       phase_poly=None, fs: float = 32e6, station_id: int = 0) -> Station:
    """codes [C, n]: padded with code 2 (+1) up to whole recording frames."""
    spf = fmt.samples_per_frame(C)
    n = codes.shape[1]
    n_pad = -(-n // spf) * spf
    full = np.full((C, n_pad), 2, dtype=np.int64)
    full[:, :n] = codes
    fr = fmt.frame_codes(torch.from_numpy(full), C, first_sample, fs, station_id)
    return Station(frames=fr, first_sample=first_sample,
                   delay_poly=np.asarray(delay_poly, dtype=np.float64),
                   phase_poly=None if phase_poly is None else np.asarray(phase_poly, np.float64),
                   station_id=station_id)


def job_from_stations(stations, *, n_chan, n_frames, sub_start, C=1, n_subbands=1,
                      n_pols=1, fs=32e6, lo_hz=None, stream_map=None) -> Job:
    if lo_hz is None:
        lo_hz = [4.82e9 + sb * fs / 2 for sb in range(n_subbands)]
    if stream_map is None:
        stream_map = list(range(n_subbands * n_pols))
    return Job(n_stations=len(stations), n_subbands=n_subbands, n_pols=n_pols, n_chan=n_chan,
               n_streams=C, stream_map=stream_map, fs_hz=fs, lo_hz=list(lo_hz),
               sub_start=sub_start, n_frames=n_frames, stations=list(stations))


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b|| / ||b|| along the last axis (max over leading axes)."""
    num = np.linalg.norm(np.asarray(a) - np.asarray(b), axis=-1)
    den = np.linalg.norm(np.asarray(b), axis=-1)
    return float(np.max(num / np.maximum(den, 1e-300)))
