"""Plain records describing one correlation job (a sub-integration).

Field meanings mirror the C-ABI's setup/station structures.  Times are in
seconds since the delay-polynomial epoch; sample indices count samples at
fs_hz since that epoch (reference time for the sub-integration, station time
for a station's recording).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Any, List, Optional, Tuple

import numpy as np


@dataclass
class Station:
    frames: Any                       # int32 [n_frames_m5b, 2504]: torch tensor or numpy array
    first_sample: int                 # station sample index of the first payload sample
    delay_poly: np.ndarray            # float64 [deg+1]: tau(t) in seconds, t = reference time
    phase_poly: Optional[np.ndarray] = None   # float64 [n_subbands, deg+1]: fringe phase in turns
    poly_span: Tuple[float, float] = (0.0, 120.0)
    station_id: int = 0
    rate_correct: bool = False        # correct the delay's drift inside each frame (O11)

    @property
    def n_frames_m5b(self) -> int:
        return int(self.frames.shape[0])


@dataclass
class Job:
    n_stations: int
    n_subbands: int
    n_pols: int
    n_chan: int
    n_streams: int                    # C, recorded streams per frame word
    stream_map: List[int]             # [n_subbands * n_pols] -> recorded stream index
    fs_hz: float
    lo_hz: List[float]                # [n_subbands] sky frequency of each band's lower edge
    sub_start: int                    # reference sample index of the sub-int start
    n_frames: int                     # FFT frames in the sub-int
    stations: List[Station] = field(default_factory=list)
    name: str = ""

    @property
    def N(self) -> int:
        return 2 * self.n_chan

    @property
    def M(self) -> int:
        return self.n_stations * self.n_pols

    @property
    def n_baselines(self) -> int:
        return self.M * (self.M + 1) // 2

    @property
    def station_samples(self) -> int:
        """Station-samples the job correlates (all frames counted)."""
        return self.n_stations * self.n_subbands * self.n_pols * self.n_frames * self.N


def baseline_index(i: int, j: int, M: int) -> int:
    """Row-major packed upper triangle (diagonal included) index of pair i <= j."""
    assert 0 <= i <= j < M
    return i * M - i * (i - 1) // 2 + (j - i)
