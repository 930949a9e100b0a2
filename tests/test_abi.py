"""C-ABI checks that need no GPU: the library loads, exports every function
include/xcorr.h declares, and the binding's ctypes structures match the C
layout (sizes and offsets printed by a C program built with gcc)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1502_06894_amd import xcorr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xcorr.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = xcorr.load_library()
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layout_matches_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "xcorr.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m))
int main(void) {
  printf("xc_setup %zu\nxc_station %zu\nxc_output %zu\n", sizeof(xc_setup), sizeof(xc_station),
         sizeof(xc_output));
  F(xc_setup, n_stations); F(xc_setup, stream_map); F(xc_setup, fs_hz); F(xc_setup, lo_hz);
  F(xc_setup, sub_start); F(xc_setup, n_frames); F(xc_setup, precision);
  F(xc_setup, frames_per_block);
  F(xc_station, frames); F(xc_station, n_frames_m5b); F(xc_station, first_sample);
  F(xc_station, frame_ok); F(xc_station, poly_deg); F(xc_station, delay_poly);
  F(xc_station, phase_poly); F(xc_station, poly_t0); F(xc_station, poly_t1);
  F(xc_station, rate_correct);
  F(xc_output, vis); F(xc_output, weight);
  printf("xc_tuning %zu\nxc_job %zu\nxc_server_stats %zu\n", sizeof(xc_tuning),
         sizeof(xc_job), sizeof(xc_server_stats));
  F(xc_tuning, fstage_waves_per_simd); F(xc_tuning, xmac_frames_per_stage);
  F(xc_tuning, xmac_channels_per_wg); F(xc_tuning, frames_per_block);
  F(xc_tuning, xmac_tiles_per_wg); F(xc_tuning, block_overlap);
  F(xc_job, setup); F(xc_job, st); F(xc_job, out);
  F(xc_server_stats, p50_ms); F(xc_server_stats, completed); F(xc_server_stats, queued);
  F(xc_server_stats, station_samples_per_s);
  printf("xc_fringe_setup %zu\nxc_fringe_peak %zu\n", sizeof(xc_fringe_setup),
         sizeof(xc_fringe_peak));
  F(xc_fringe_setup, n_subints); F(xc_fringe_setup, rate_win); F(xc_fringe_setup, chan_width_hz);
  F(xc_fringe_setup, t_int_s);
  F(xc_fringe_peak, delay_bin); F(xc_fringe_peak, amp); F(xc_fringe_peak, rate_off);
  F(xc_fringe_peak, delay_s); F(xc_fringe_peak, rate_hz);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)],
                   check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True,
                                                       text=True, check=True).stdout.splitlines())
    py = {"xc_setup": xcorr.XcSetup, "xc_station": xcorr.XcStation, "xc_output": xcorr.XcOutput,
          "xc_tuning": xcorr.XcTuning, "xc_job": xcorr.XcJob,
          "xc_server_stats": xcorr.XcServerStats, "xc_fringe_setup": xcorr.XcFringeSetup,
          "xc_fringe_peak": xcorr.XcFringePeak}
    for key, val in out.items():
        if "." in key:
            t, m = key.split(".")
            assert getattr(py[t], m).offset == int(val), key
        else:
            assert C.sizeof(py[key]) == int(val), key


def test_strerror_codes():
    assert xcorr.strerror(0) == "ok"
    assert "workspace" in xcorr.strerror(xcorr.XC_E_NOMEM)
    assert xcorr.strerror(-99) == "unknown error"


def _setup(**kw):
    sm = (C.c_int32 * 32)(*range(32))
    lo = (C.c_double * 16)(*([4.82e9] * 16))
    s = xcorr.XcSetup(2, 1, 1, 256, 1, C.cast(sm, C.POINTER(C.c_int32)), 32e6,
                      C.cast(lo, C.POINTER(C.c_double)), 37 * 32_000_000, 100, 0, 0)
    for k, v in kw.items():
        setattr(s, k, v)
    poly = (C.c_double * 6)(0.4, 1e-5, 0, 0, 0, 0)
    st = (xcorr.XcStation * 2)()
    for i in range(2):
        st[i] = xcorr.XcStation(0x1000, 10, 0, None, 5, C.cast(poly, C.POINTER(C.c_double)),
                                None, 0.0, 120.0)
    return s, st, (sm, lo, poly)


def test_workspace_bytes_and_validation_on_host():
    lib = xcorr.load_library()
    s, st, keep = _setup()
    n = lib.xc_workspace_bytes(None, C.byref(s), st)
    assert n > 256 * 2 * 100 * 8          # at least the staged spectra
    s2, st2, keep2 = _setup(frames_per_block=32)   # two 32-frame block buffers < 100 frames
    assert lib.xc_workspace_bytes(None, C.byref(s2), st2) < n
    for bad in [dict(n_chan=300), dict(n_chan=64), dict(n_streams_recorded=3),
                dict(n_pols=3), dict(n_stations=0), dict(n_frames=0), dict(frames_per_block=70000),
                dict(precision=7)]:
        sb, stb, kb = _setup(**bad)
        assert lib.xc_workspace_bytes(None, C.byref(sb), stb) == 0, bad
    # the default block of a small job: past 2048 frames while its spectra stay
    # within 16 GiB (here the whole 10000-frame job in one block)
    s4, st4, k4 = _setup(n_frames=10000)
    s5, st5, k5 = _setup(n_frames=10000, frames_per_block=2048)
    s6, st6, k6 = _setup(n_frames=10000, frames_per_block=10000)
    n4 = lib.xc_workspace_bytes(None, C.byref(s4), st4)
    assert n4 > lib.xc_workspace_bytes(None, C.byref(s5), st5)
    assert n4 == lib.xc_workspace_bytes(None, C.byref(s6), st6)
    # sub-integration outside the polynomial span
    s3, st3, k3 = _setup(sub_start=200 * 32_000_000)
    assert lib.xc_workspace_bytes(None, C.byref(s3), st3) == 0


def test_fringe_workspace_and_validation_on_host():
    lib = xcorr.load_library()

    def fs(**kw):
        d = dict(n_subints=8, n_subbands=2, n_baselines=3, n_chan=128, delay_len=256, rate_len=16,
                 delay_win=0, rate_win=0, chan_width_hz=1e4, t_int_s=0.5)
        d.update(kw)
        return xcorr.XcFringeSetup(**d)
    n = lib.xc_fringe_workspace_bytes(C.byref(fs()))
    assert n >= 2 * 3 * 8 * 256 * 8                       # the delay-transform rows
    assert xcorr.FRINGE_PEAK_DTYPE.itemsize == C.sizeof(xcorr.XcFringePeak)
    for bad in [dict(delay_len=300), dict(delay_len=128), dict(n_chan=512), dict(rate_len=4),
                dict(rate_len=2048), dict(n_subints=0), dict(n_subints=300, rate_len=512),
                dict(t_int_s=0.0), dict(delay_win=-1)]:
        assert lib.xc_fringe_workspace_bytes(C.byref(fs(**bad))) == 0, bad


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    ctx = C.c_void_p()
    assert xcorr.load_library().xc_create(C.byref(ctx), 0) == xcorr.XC_E_HIP
