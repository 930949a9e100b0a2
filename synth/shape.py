"""Shape-only generator: recordings with the right sizes, code statistics and
a shared sky component, built with torch on any device (CPU for tests, the GPU
for full-size workloads).

Station s, stream c, station sample j records
    sqrt(rho) * sky_c[j - shift_s] + sqrt(1 - rho) * noise_{s,c}[j]
quantised to 2 bits.  sky_c is white Gaussian noise indexed by reference
sample; the integer shift_s plays the role of the station's delay.  The
generated voltages carry no fringe phase, so jobs built here are correlated
either with delay models matched to the shifts (constant polynomials
shift_s / fs, zero phase) or, for timing, with realistic polynomials against
which the data are just noise.

Random numbers come from torch generators seeded per (purpose, block) with
SplitMix64-mixed seeds, so any sample range is reproducible on a given device.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import format as fmt
from .job import Job, Station
from .physics import seed_of

SKY_BLOCK = 1 << 22


class _Sky:
    """Shared sky streams, generated in fixed blocks of the reference index."""

    def __init__(self, C: int, seed: int, device, cache: int = 4):
        self.C, self.seed, self.device, self.cache = C, seed, device, cache
        self._blocks: dict = {}

    def _block(self, b: int) -> torch.Tensor:
        if b not in self._blocks:
            if len(self._blocks) >= self.cache:
                self._blocks.pop(next(iter(self._blocks)))
            g = torch.Generator(device=self.device).manual_seed(seed_of(self.seed, 0x5C1, b))
            self._blocks[b] = torch.randn(self.C, SKY_BLOCK, generator=g, device=self.device)
        return self._blocks[b]

    def range(self, r0: int, L: int) -> torch.Tensor:
        b0, b1 = r0 // SKY_BLOCK, (r0 + L - 1) // SKY_BLOCK
        parts = [self._block(b) for b in range(b0, b1 + 1)]
        cat = parts[0] if len(parts) == 1 else torch.cat(parts, dim=1)
        off = r0 - b0 * SKY_BLOCK
        return cat[:, off:off + L]


def make_station_frames(*, C: int, fs: float, first_sample: int, n_m5b: int,
                        shift: int, station_id: int, sky: _Sky, seed: int, rho: float,
                        device, chunk_frames: Optional[int] = None) -> torch.Tensor:
    spf = fmt.samples_per_frame(C)
    if chunk_frames is None:
        chunk_frames = max(1, (1 << 22) // spf)
    frames = torch.empty(n_m5b, fmt.FRAME_WORDS, dtype=torch.int32, device=device)
    a, b = math.sqrt(rho), math.sqrt(1.0 - rho)
    for f0 in range(0, n_m5b, chunk_frames):
        nf = min(chunk_frames, n_m5b - f0)
        L = nf * spf
        j0 = first_sample + f0 * spf
        g = torch.Generator(device=device).manual_seed(seed_of(seed, 0x401, station_id, f0))
        x = torch.randn(C, L, generator=g, device=device).mul_(b)
        x.add_(sky.range(j0 - shift, L), alpha=a)
        codes = fmt.quantise(x)
        del x
        frames[f0:f0 + nf, :fmt.HEADER_WORDS] = fmt.headers(nf, C, first_sample, fs,
                                                            station_id, device, frame0=f0)
        frames[f0:f0 + nf, fmt.HEADER_WORDS:] = fmt.pack_codes(codes, C).reshape(nf, fmt.PAYLOAD_WORDS)
        del codes
    return frames


def build_job(*, n_stations: int, n_subbands: int, n_pols: int, n_chan: int, C: int,
              fs: float, lo_hz: Sequence[float], sub_start: int, n_frames: int,
              delay_polys: List[Sequence[float]], shifts: Sequence[int],
              phase_zero: bool, seed: int, rho: float = 0.05, device="cpu",
              margin: int = 4096, stream_map: Optional[List[int]] = None,
              poly_span=(0.0, 120.0), name: str = "") -> Job:
    """Job whose stations record the shared sky at the given integer shifts."""
    from .physics import buffer_extent
    N = 2 * n_chan
    if stream_map is None:
        stream_map = [sb * n_pols + p for sb in range(n_subbands) for p in range(n_pols)]
    assert max(stream_map) < C
    sky = _Sky(C, seed, device)
    stations = []
    for s in range(n_stations):
        first, n_m5b = buffer_extent(delay_polys[s], sub_start, n_frames, N, fs, C, margin)
        fr = make_station_frames(C=C, fs=fs, first_sample=first, n_m5b=n_m5b,
                                 shift=int(shifts[s]), station_id=s, sky=sky, seed=seed,
                                 rho=rho, device=device)
        deg = len(delay_polys[s]) - 1
        pp = np.zeros((n_subbands, deg + 1)) if phase_zero else None
        stations.append(Station(frames=fr, first_sample=first,
                                delay_poly=np.asarray(delay_polys[s], dtype=np.float64),
                                phase_poly=pp, poly_span=poly_span, station_id=s))
    return Job(n_stations=n_stations, n_subbands=n_subbands, n_pols=n_pols, n_chan=n_chan,
               n_streams=C, stream_map=list(stream_map), fs_hz=fs, lo_hz=list(lo_hz),
               sub_start=sub_start, n_frames=n_frames, stations=stations, name=name)
