"""Mark5B-style recording format used throughout this repository (packer side).

The paper converts RadioAstron's native recordings to Mark5B so that the
correlator can read them (section 2, data-format paragraph), but the Mark5B
manual is not part of the material, so this repository fixes its own format:

  * a frame is 10016 bytes: a 16-byte header (4 little-endian uint32 words)
    followed by a 10000-byte payload (2500 little-endian uint32 words);
  * header word 0 is the sync word 0xABADDEED, word 1 is the frame number
    within the second (bits 0-14) OR'ed with the station id shifted left by 16,
    word 2 is the integer second since the polynomial epoch, word 3 is zero;
  * with C recorded streams (C in {1, 2, 4, 8, 16}) each payload word carries
    16 two-bit fields; field j (bits 2j, 2j+1) is stream (j mod C) at
    per-stream sample index  word * (16 / C) + floor(j / C), where "word"
    counts payload words from the start of the recording;
  * codes are offset binary: 0, 1, 2, 3 stand for -3.3359, -1, +1, +3.3359.

Only the sync word is inspected by the correlator; the other header words are
informational.  This module writes the format; the oracle and the GPU library
each read it with their own code.
"""
from __future__ import annotations

import numpy as np
import torch

SYNC_WORD = 0xABADDEED
HEADER_WORDS = 4
PAYLOAD_WORDS = 2500
FRAME_WORDS = HEADER_WORDS + PAYLOAD_WORDS      # 2504
FRAME_BYTES = 4 * FRAME_WORDS                   # 10016
FIELDS_PER_WORD = 16
VALID_C = (1, 2, 4, 8, 16)

# two-bit quantiser thresholds in units of sigma (optimum 4-level quantiser)
QUANT_THRESHOLD = 0.9816


def samples_per_frame(C: int) -> int:
    """Per-stream samples carried by one frame's payload."""
    if C not in VALID_C:
        raise ValueError(f"C={C} not in {VALID_C}")
    return PAYLOAD_WORDS * FIELDS_PER_WORD // C


def quantise(x: torch.Tensor, sigma: float = 1.0) -> torch.Tensor:
    """2-bit offset-binary codes of real samples (thresholds -t, 0, +t)."""
    t = QUANT_THRESHOLD * sigma
    return ((x >= -t).to(torch.int64) + (x >= 0).to(torch.int64)
            + (x >= t).to(torch.int64))


def _u32_to_i32(w: torch.Tensor) -> torch.Tensor:
    return torch.where(w >= 2**31, w - 2**32, w).to(torch.int32)


def pack_codes(codes: torch.Tensor, C: int) -> torch.Tensor:
    """Pack codes [C, n] (n a multiple of 16/C) into payload words (int32 [n*C/16]).

    The int32 values are the uint32 words' bit patterns.
    """
    Cc, n = codes.shape
    assert Cc == C, (Cc, C)
    spw = FIELDS_PER_WORD // C
    assert n % spw == 0, (n, spw)
    # [C, n_words, spw] -> [n_words, spw, C] -> [n_words, 16]; field j = sub*C + c
    f = codes.to(torch.int64).reshape(C, n // spw, spw).permute(1, 2, 0)
    f = f.reshape(n // spw, FIELDS_PER_WORD)
    shifts = 2 * torch.arange(FIELDS_PER_WORD, device=codes.device, dtype=torch.int64)
    words = (f << shifts).sum(dim=1)
    return _u32_to_i32(words)


def headers(n_frames: int, C: int, first_sample: int, fs_hz: float,
            station_id: int, device="cpu", frame0: int = 0) -> torch.Tensor:
    """Header words (int32 [n_frames, 4]) for frames frame0 .. frame0+n_frames-1."""
    spf = samples_per_frame(C)
    fs_int = int(round(fs_hz))
    fm = torch.arange(frame0, frame0 + n_frames, dtype=torch.int64, device=device)
    s0 = first_sample + fm * spf
    sec = torch.div(s0, fs_int, rounding_mode="floor")
    fr = torch.div(s0 - sec * fs_int, spf, rounding_mode="floor")
    h = torch.zeros(n_frames, HEADER_WORDS, dtype=torch.int64, device=device)
    h[:, 0] = SYNC_WORD
    h[:, 1] = (fr & 0x7FFF) | (int(station_id) << 16)
    h[:, 2] = sec & 0xFFFFFFFF
    return _u32_to_i32(h)


def frame_codes(codes: torch.Tensor, C: int, first_sample: int, fs_hz: float,
                station_id: int) -> torch.Tensor:
    """Codes [C, n] (n a multiple of samples_per_frame) -> frames int32 [n_frames, 2504]."""
    spf = samples_per_frame(C)
    n = codes.shape[1]
    assert n % spf == 0, (n, spf)
    nf = n // spf
    out = torch.empty(nf, FRAME_WORDS, dtype=torch.int32, device=codes.device)
    out[:, :HEADER_WORDS] = headers(nf, C, first_sample, fs_hz, station_id, codes.device)
    out[:, HEADER_WORDS:] = pack_codes(codes, C).reshape(nf, PAYLOAD_WORDS)
    return out


def as_u32(frames) -> np.ndarray:
    """View an int32 frames tensor/array as numpy uint32 (host copy if on device)."""
    if isinstance(frames, torch.Tensor):
        frames = frames.detach().cpu().numpy()
    return np.ascontiguousarray(frames).view(np.uint32)
