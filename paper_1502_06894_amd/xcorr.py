"""ctypes binding of libxcorr.so (include/xcorr.h): argument marshalling only.

Every step of the correlation runs in the library's HIP kernels.  torch is
used for device memory and the current stream; there is no fallback: if the
library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libxcorr.so")

XC_OK, XC_E_INVAL, XC_E_RANGE, XC_E_NOMEM, XC_E_HIP, XC_E_CANCELLED, XC_E_TIMEOUT = (
    0, -1, -2, -3, -4, -5, -6)
XC_FP32, XC_FP16_MFMA, XC_FP8_MFMA = 0, 1, 2
KERNEL_KINDS = ["ingest", "delays", "fstage", "xmac", "xmfma", "finalise", "zero", "fringe",
                "feed"]
PRECISIONS = {"fp32": XC_FP32, "fp16": XC_FP16_MFMA, "fp8": XC_FP8_MFMA}


class XcSetup(C.Structure):
    _fields_ = [("n_stations", C.c_int32), ("n_subbands", C.c_int32), ("n_pols", C.c_int32),
                ("n_chan", C.c_int32), ("n_streams_recorded", C.c_int32),
                ("stream_map", C.POINTER(C.c_int32)), ("fs_hz", C.c_double),
                ("lo_hz", C.POINTER(C.c_double)), ("sub_start", C.c_int64),
                ("n_frames", C.c_int64), ("precision", C.c_int32),
                ("frames_per_block", C.c_int32)]


class XcStation(C.Structure):
    _fields_ = [("frames", C.c_void_p), ("n_frames_m5b", C.c_int64),
                ("first_sample", C.c_int64), ("frame_ok", C.c_void_p),
                ("poly_deg", C.c_int32), ("delay_poly", C.POINTER(C.c_double)),
                ("phase_poly", C.POINTER(C.c_double)), ("poly_t0", C.c_double),
                ("poly_t1", C.c_double), ("rate_correct", C.c_int32)]


class XcOutput(C.Structure):
    _fields_ = [("vis", C.c_void_p), ("weight", C.c_void_p)]


class XcJob(C.Structure):
    _fields_ = [("setup", XcSetup), ("st", C.POINTER(XcStation)), ("out", XcOutput)]


XC_BATCH_GRAPH = 1
XC_BATCH_LANES = 2
# xc_tuning.xmac_frames_per_stage: FP32 products on the matrix cores
XMAC_MATRIX = 3
# ... the same products fed through the LDS ring
XMAC_MATRIX_RING = 5


class XcTuning(C.Structure):
    _fields_ = [("fstage_waves_per_simd", C.c_int32), ("xmac_frames_per_stage", C.c_int32),
                ("xmac_channels_per_wg", C.c_int32), ("frames_per_block", C.c_int32),
                ("xmac_tiles_per_wg", C.c_int32), ("block_overlap", C.c_int32)]


class XcFringeSetup(C.Structure):
    _fields_ = [("n_subints", C.c_int32), ("n_subbands", C.c_int32), ("n_baselines", C.c_int32),
                ("n_chan", C.c_int32), ("delay_len", C.c_int32), ("rate_len", C.c_int32),
                ("delay_win", C.c_int32), ("rate_win", C.c_int32),
                ("chan_width_hz", C.c_double), ("t_int_s", C.c_double)]


class XcFringePeak(C.Structure):
    _fields_ = [("delay_bin", C.c_int32), ("rate_bin", C.c_int32), ("amp", C.c_float),
                ("phase", C.c_float), ("delay_off", C.c_float), ("rate_off", C.c_float),
                ("delay_s", C.c_double), ("rate_hz", C.c_double)]


# numpy view of an xc_fringe_peak array
FRINGE_PEAK_DTYPE = np.dtype([("delay_bin", "<i4"), ("rate_bin", "<i4"), ("amp", "<f4"),
                              ("phase", "<f4"), ("delay_off", "<f4"), ("rate_off", "<f4"),
                              ("delay_s", "<f8"), ("rate_hz", "<f8")])


class XcFeedSetup(C.Structure):
    _fields_ = [("n_subints", C.c_int32), ("n_subbands", C.c_int32), ("n_stations", C.c_int32),
                ("n_chan", C.c_int32), ("feed", C.c_int32)]


XC_FEED_CIRCULAR, XC_FEED_LINEAR = 0, 1


class XcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"xcorr error {code}: {msg}")
        self.code = code


_lib = None


def load_library() -> C.CDLL:
    """Load libxcorr.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is not built (run __graft_entry__.build())")
        lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        sig = {
            "xc_create": (C.c_int, [C.POINTER(P), C.c_int]),
            "xc_destroy": (None, [P]),
            "xc_strerror": (C.c_char_p, [C.c_int]),
            "xc_last_error": (C.c_char_p, [P]),
            "xc_ingest": (C.c_int, [P, P, C.c_int64, P, P]),
            "xc_validate": (C.c_int, [P, C.POINTER(XcSetup), C.POINTER(XcStation)]),
            "xc_workspace_bytes": (C.c_size_t, [P, C.POINTER(XcSetup), C.POINTER(XcStation)]),
            "xc_correlate_subint": (C.c_int, [P, C.POINTER(XcSetup), C.POINTER(XcStation),
                                              C.POINTER(XcOutput), P, C.c_size_t, P]),
            "xc_correlate_subint_noalloc": (C.c_int, [P, C.POINTER(XcSetup), C.POINTER(XcStation),
                                                      C.POINTER(XcOutput), P]),
            "xc_noalloc_scratch_bytes": (C.c_size_t, []),
            "xc_debug_delays": (C.c_int, [P, C.POINTER(XcSetup), C.POINTER(XcStation), P, P, P, P,
                                          P, C.c_size_t, P]),
            "xc_debug_unpack": (C.c_int, [P, C.POINTER(XcSetup), C.POINTER(XcStation), C.c_int32,
                                          C.c_int32, C.c_int64, P, P, C.c_size_t, P]),
            "xc_debug_spectra": (C.c_int, [P, C.POINTER(XcSetup), C.POINTER(XcStation),
                                           C.c_int64, C.c_int32, P, P, C.c_size_t, P]),
            "xc_batch_workspace_bytes": (C.c_size_t, [P, C.POINTER(XcJob), C.c_int32, C.c_int32,
                                                      C.c_int32]),
            "xc_correlate_batch": (C.c_int, [P, C.POINTER(XcJob), C.c_int32, C.c_int32, C.c_int32,
                                             P, C.c_size_t, P]),
            "xc_autotune": (C.c_int, [P, C.POINTER(XcSetup), C.POINTER(XcStation),
                                      C.POINTER(XcOutput), P, C.c_size_t, P,
                                      C.POINTER(XcTuning)]),
            "xc_set_tuning": (C.c_int, [P, C.POINTER(XcTuning)]),
            "xc_get_tuning": (C.c_int, [P, C.POINTER(XcTuning)]),
            "xc_fringe_workspace_bytes": (C.c_size_t, [C.POINTER(XcFringeSetup)]),
            "xc_fringe_search": (C.c_int, [P, C.POINTER(XcFringeSetup), P, P, P, P, C.c_size_t,
                                           P]),
            "xc_feed_correct": (C.c_int, [P, C.POINTER(XcFeedSetup), P, P, P]),
            "xc_profile_begin": (C.c_int, [P, C.c_int32]),
            "xc_profile_end": (C.c_int, [P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    return load_library().xc_strerror(code).decode()


class _Marshal:
    """ctypes views of a Job (keeps the host arrays alive for the call)."""

    def __init__(self, job, precision: int = XC_FP32, frames_per_block: int = 0,
                 frame_ok: Optional[Sequence] = None):
        self.keep = []
        sm = np.ascontiguousarray(job.stream_map, dtype=np.int32)
        lo = np.ascontiguousarray(job.lo_hz, dtype=np.float64)
        self.keep += [sm, lo]
        self.setup = XcSetup(job.n_stations, job.n_subbands, job.n_pols, job.n_chan,
                             job.n_streams, sm.ctypes.data_as(C.POINTER(C.c_int32)),
                             float(job.fs_hz), lo.ctypes.data_as(C.POINTER(C.c_double)),
                             int(job.sub_start), int(job.n_frames), int(precision),
                             int(frames_per_block))
        arr = (XcStation * job.n_stations)()
        for i, st in enumerate(job.stations):
            fr = st.frames
            if not (isinstance(fr, torch.Tensor) and fr.is_cuda and fr.dtype == torch.int32
                    and fr.is_contiguous() and fr.dim() == 2 and fr.shape[1] == 2504):
                raise ValueError(f"station {i}: frames must be a contiguous cuda int32 [n, 2504]")
            dp = np.ascontiguousarray(st.delay_poly, dtype=np.float64)
            self.keep.append(dp)
            pp_ptr = None
            if st.phase_poly is not None:
                pp = np.ascontiguousarray(st.phase_poly, dtype=np.float64)
                assert pp.shape == (job.n_subbands, dp.shape[0]), pp.shape
                self.keep.append(pp)
                pp_ptr = pp.ctypes.data_as(C.POINTER(C.c_double))
            ok = None
            if frame_ok is not None and frame_ok[i] is not None:
                ok = frame_ok[i].data_ptr()
            arr[i] = XcStation(fr.data_ptr(), fr.shape[0], int(st.first_sample), ok,
                               dp.shape[0] - 1, dp.ctypes.data_as(C.POINTER(C.c_double)),
                               pp_ptr, float(st.poly_span[0]), float(st.poly_span[1]),
                               int(bool(getattr(st, "rate_correct", False))))
        self.stations = arr


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Correlator:
    """One library context on a HIP device."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        self.ctx = C.c_void_p()
        rc = self.lib.xc_create(C.byref(self.ctx), device)
        if rc != XC_OK:
            raise XcError(rc, strerror(rc))

    def close(self):
        if self.ctx:
            self.lib.xc_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != XC_OK:
            raise XcError(rc, f"{strerror(rc)}: {self.lib.xc_last_error(self.ctx).decode()}")

    # ------------------------------------------------------------------ sizes
    def workspace_bytes(self, job, precision: int = XC_FP32, frames_per_block: int = 0,
                        frame_ok=None) -> int:
        m = _Marshal(job, precision, frames_per_block, frame_ok)
        self._check(self.lib.xc_validate(self.ctx, C.byref(m.setup), m.stations))
        return int(self.lib.xc_workspace_bytes(self.ctx, C.byref(m.setup), m.stations))

    def alloc_workspace(self, job, **kw) -> torch.Tensor:
        n = self.workspace_bytes(job, **kw)
        if n == 0:
            raise XcError(XC_E_INVAL, "invalid job (workspace size 0)")
        return torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")

    def alloc_output(self, job):
        dev = f"cuda:{self.device}"
        vis = torch.empty(job.n_subbands, job.n_baselines, job.n_chan, dtype=torch.complex64,
                          device=dev)
        w = torch.empty(job.n_subbands, job.n_baselines, dtype=torch.float32, device=dev)
        return vis, w

    # ------------------------------------------------------------------ calls
    def ingest(self, frames: torch.Tensor, frame_ok: Optional[torch.Tensor] = None,
               stream=None) -> torch.Tensor:
        if frame_ok is None:
            frame_ok = torch.empty(frames.shape[0], dtype=torch.uint8, device=frames.device)
        self._check(self.lib.xc_ingest(self.ctx, frames.data_ptr(), frames.shape[0],
                                       frame_ok.data_ptr(), _stream_ptr(stream)))
        return frame_ok

    def correlate(self, job, *, precision: int = XC_FP32, frames_per_block: int = 0,
                  out=None, workspace: Optional[torch.Tensor] = None, stream=None,
                  frame_ok=None):
        """Returns (vis complex64 [n_sb, nbl, n_chan], weight float32 [n_sb, nbl])."""
        m = _Marshal(job, precision, frames_per_block, frame_ok)
        if workspace is None:
            workspace = self.alloc_workspace(job, precision=precision,
                                             frames_per_block=frames_per_block, frame_ok=frame_ok)
        vis, w = out if out is not None else self.alloc_output(job)
        o = XcOutput(vis.data_ptr(), w.data_ptr())
        self._check(self.lib.xc_correlate_subint(self.ctx, C.byref(m.setup), m.stations,
                                                 C.byref(o), workspace.data_ptr(),
                                                 workspace.numel(), _stream_ptr(stream)))
        return vis, w

    def correlate_noalloc(self, job, *, precision: int = XC_FP32, frames_per_block: int = 0,
                          out=None, stream=None, frame_ok=None):
        """As correlate(), in the library's fixed device scratch (no workspace)."""
        m = _Marshal(job, precision, frames_per_block, frame_ok)
        vis, w = out if out is not None else self.alloc_output(job)
        o = XcOutput(vis.data_ptr(), w.data_ptr())
        self._check(self.lib.xc_correlate_subint_noalloc(self.ctx, C.byref(m.setup), m.stations,
                                                         C.byref(o), _stream_ptr(stream)))
        return vis, w

    # ------------------------------------------------------------------ batches
    def _batch_structs(self, jobs, precision, outs):
        ms = [_Marshal(j, precision) for j in jobs]
        if outs is None:
            outs = [self.alloc_output(j) for j in jobs]
        arr = (XcJob * len(jobs))()
        for i, (m, (vis, w)) in enumerate(zip(ms, outs)):
            arr[i] = XcJob(m.setup, C.cast(m.stations, C.POINTER(XcStation)),
                           XcOutput(vis.data_ptr(), w.data_ptr()))
        return ms, outs, arr

    def correlate_batch(self, jobs, *, n_lanes: int = 4, graph: bool = False,
                        lanes_only: bool = False, precision=XC_FP32, outs=None,
                        workspace: Optional[torch.Tensor] = None, stream=None):
        """Correlate a list of jobs as one batch; returns [(vis, weight), ...].

        Default: the fused executor (one persistent F-stage launch per FFT length
        and round); lanes_only: every job as a single job on the lanes.
        precision: one value for all jobs, or a list with one per job."""
        if not isinstance(precision, (list, tuple)):
            precision = [precision] * len(jobs)
        flags = (XC_BATCH_GRAPH if graph else 0) | (XC_BATCH_LANES if lanes_only else 0)
        ms = [_Marshal(j, p) for j, p in zip(jobs, precision)]
        if outs is None:
            outs = [self.alloc_output(j) for j in jobs]
        arr = (XcJob * len(jobs))()
        for i, (m, (vis, w)) in enumerate(zip(ms, outs)):
            arr[i] = XcJob(m.setup, C.cast(m.stations, C.POINTER(XcStation)),
                           XcOutput(vis.data_ptr(), w.data_ptr()))
        if workspace is None:
            n = int(self.lib.xc_batch_workspace_bytes(self.ctx, arr, len(jobs), n_lanes, flags))
            if n == 0:   # invalid job: the batch call itself reports which and why
                self._check(self.lib.xc_correlate_batch(self.ctx, arr, len(jobs), n_lanes, flags,
                                                        None, 0, None))
            workspace = torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")
        self._check(self.lib.xc_correlate_batch(self.ctx, arr, len(jobs), n_lanes, flags,
                                                workspace.data_ptr(), workspace.numel(),
                                                _stream_ptr(stream)))
        return outs

    def batch_workspace(self, jobs, n_lanes: int = 4, precision=XC_FP32,
                        lanes_only: bool = False) -> torch.Tensor:
        if not isinstance(precision, (list, tuple)):
            precision = [precision] * len(jobs)
        flags = XC_BATCH_LANES if lanes_only else 0
        ms = [_Marshal(j, p) for j, p in zip(jobs, precision)]
        arr = (XcJob * len(jobs))()
        for i, m in enumerate(ms):
            arr[i] = XcJob(m.setup, C.cast(m.stations, C.POINTER(XcStation)), XcOutput(1, 1))
        n = int(self.lib.xc_batch_workspace_bytes(self.ctx, arr, len(jobs), n_lanes, flags))
        if n == 0:
            self._check(self.lib.xc_correlate_batch(self.ctx, arr, len(jobs), n_lanes, flags, None,
                                                    0, None))
        return torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")

    def autotune(self, job, *, precision=XC_FP32, workspace: Optional[torch.Tensor] = None,
                 stream=None) -> dict:
        """Time launch-shape candidates on `job` and cache the best for its shape."""
        m = _Marshal(job, precision)
        if workspace is None:
            saved = self.get_tuning()
            self.set_tuning(frames_per_block=2048)
            try:
                workspace = self.alloc_workspace(job, precision=precision)
            finally:
                self.set_tuning(**saved)
        vis, w = self.alloc_output(job)
        t = XcTuning()
        self._check(self.lib.xc_autotune(self.ctx, C.byref(m.setup), m.stations,
                                         C.byref(XcOutput(vis.data_ptr(), w.data_ptr())),
                                         workspace.data_ptr(), workspace.numel(),
                                         _stream_ptr(stream), C.byref(t)))
        return {f: getattr(t, f) for f, _ in XcTuning._fields_}

    def set_tuning(self, **kw):
        """Set launch-shape parameters (fstage_waves_per_simd, xmac_frames_per_stage,
        xmac_channels_per_wg, frames_per_block, xmac_tiles_per_wg, block_overlap);
        unspecified ones keep their value."""
        t = XcTuning()
        self._check(self.lib.xc_get_tuning(self.ctx, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        self._check(self.lib.xc_set_tuning(self.ctx, C.byref(t)))

    def get_tuning(self) -> dict:
        t = XcTuning()
        self._check(self.lib.xc_get_tuning(self.ctx, C.byref(t)))
        return {f: getattr(t, f) for f, _ in XcTuning._fields_}

    def fringe_search(self, vis: torch.Tensor, delay_len: int, rate_len: int,
                      chan_width_hz: float, t_int_s: float, delay_win: int = 0,
                      rate_win: int = 0, want_map: bool = False, workspace=None, stream=None):
        """Delay-rate fringe search (xc_fringe_search) over vis, a device complex64
        tensor [T, n_subbands, n_baselines, n_chan].  Returns (peaks, map): peaks a
        numpy structured array [n_subbands, n_baselines] (FRINGE_PEAK_DTYPE), map the
        device complex64 tensor [n_subbands, n_baselines, rate_len, delay_len] or None."""
        if vis.dtype != torch.complex64 or vis.dim() != 4 or not vis.is_cuda:
            raise XcError(XC_E_INVAL, "vis must be a 4-d complex64 device tensor")
        vis = vis.contiguous()
        T, nsb, nbl, nch = vis.shape
        fs = XcFringeSetup(T, nsb, nbl, nch, int(delay_len), int(rate_len), int(delay_win),
                           int(rate_win), float(chan_width_hz), float(t_int_s))
        need = int(self.lib.xc_fringe_workspace_bytes(C.byref(fs)))
        if need == 0:
            # let the library name what is wrong
            self._check(self.lib.xc_fringe_search(self.ctx, C.byref(fs), None, None, None, None,
                                                  0, None))
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=vis.device)
        peaks = torch.empty((nsb, nbl, FRINGE_PEAK_DTYPE.itemsize), dtype=torch.uint8,
                            device=vis.device)
        gmap = (torch.empty((nsb, nbl, rate_len, delay_len), dtype=torch.complex64,
                            device=vis.device) if want_map else None)
        self._check(self.lib.xc_fringe_search(
            self.ctx, C.byref(fs), vis.data_ptr(), peaks.data_ptr(),
            gmap.data_ptr() if gmap is not None else None, workspace.data_ptr(),
            workspace.numel(), _stream_ptr(stream)))
        (stream or torch.cuda.current_stream()).synchronize()
        out = np.frombuffer(peaks.cpu().numpy().tobytes(), dtype=FRINGE_PEAK_DTYPE)
        return out.reshape(nsb, nbl), gmap

    def feed_correct(self, vis: torch.Tensor, angles: torch.Tensor, feed: int, stream=None):
        """Feed-angle correction (xc_feed_correct), in place: vis a device complex64
        tensor [T, n_subbands, M(M+1)/2, n_chan] with M = 2 S, angles a device float64
        tensor [T, S] in radians."""
        if vis.dtype != torch.complex64 or vis.dim() != 4 or not vis.is_contiguous():
            raise XcError(XC_E_INVAL, "vis must be a contiguous 4-d complex64 device tensor")
        angles = angles.to(device=vis.device, dtype=torch.float64).contiguous()
        T, nsb, nbl, nch = vis.shape
        if angles.dim() != 2 or angles.shape[0] != T:
            raise XcError(XC_E_INVAL, "angles must be [T, S] with T = vis.shape[0]")
        S = angles.shape[1]
        if nbl != S * (2 * S + 1):
            raise XcError(XC_E_INVAL, f"vis has {nbl} products; {S} dual-pol stations give "
                                      f"{S * (2 * S + 1)}")
        fs = XcFeedSetup(T, nsb, S, nch, int(feed))
        self._check(self.lib.xc_feed_correct(self.ctx, C.byref(fs), vis.data_ptr(),
                                             angles.data_ptr(), _stream_ptr(stream)))
        return vis

    def profile_begin(self, max_launches: int = 8192):
        """Time every kernel launch of this context with HIP events on its stream."""
        self._check(self.lib.xc_profile_begin(self.ctx, max_launches))

    def profile_end(self) -> dict:
        """{kind: (total ms, launches)} since profile_begin (synchronises)."""
        ms = np.zeros(len(KERNEL_KINDS), np.float64)
        n = np.zeros(len(KERNEL_KINDS), np.int64)
        self._check(self.lib.xc_profile_end(self.ctx, ms.ctypes.data, n.ctypes.data))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_KINDS)}

    def debug_delays(self, job, workspace: Optional[torch.Tensor] = None, frames_per_block=0):
        m = _Marshal(job, XC_FP32, frames_per_block)
        if workspace is None:
            workspace = self.alloc_workspace(job, frames_per_block=frames_per_block)
        S, F, nsb = job.n_stations, job.n_frames, job.n_subbands
        n_int = np.zeros((S, F), np.int64)
        d = np.zeros((S, F), np.float64)
        valid = np.zeros((S, F), np.int32)
        phi0 = np.zeros((S, nsb, F), np.float64)
        self._check(self.lib.xc_debug_delays(
            self.ctx, C.byref(m.setup), m.stations, n_int.ctypes.data, d.ctypes.data,
            valid.ctypes.data, phi0.ctypes.data, workspace.data_ptr(), workspace.numel(),
            _stream_ptr(None)))
        return dict(n_int=n_int, d=d, valid=valid.astype(bool), phi0=phi0)

    def debug_unpack(self, job, station: int, inp: int, frame: int,
                     workspace: Optional[torch.Tensor] = None) -> np.ndarray:
        m = _Marshal(job)
        if workspace is None:
            workspace = self.alloc_workspace(job)
        out = np.zeros(job.N, np.float32)
        self._check(self.lib.xc_debug_unpack(self.ctx, C.byref(m.setup), m.stations, station,
                                             inp, frame, out.ctypes.data, workspace.data_ptr(),
                                             workspace.numel(), _stream_ptr(None)))
        return out

    def debug_spectra(self, job, frame0: int, n: int, frames_per_block: int = 0,
                      workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Spectra after the F stage: complex64 [n_sb, n, M, n_chan]."""
        m = _Marshal(job, XC_FP32, frames_per_block)
        if workspace is None:
            workspace = self.alloc_workspace(job, frames_per_block=frames_per_block)
        spec = torch.empty(job.n_subbands, n, job.M, job.n_chan, dtype=torch.complex64,
                           device=f"cuda:{self.device}")
        self._check(self.lib.xc_debug_spectra(self.ctx, C.byref(m.setup), m.stations, frame0, n,
                                              spec.data_ptr(), workspace.data_ptr(),
                                              workspace.numel(), _stream_ptr(None)))
        return spec


def job_to_device(job, device="cuda:0"):
    """Copy a job's recordings to the GPU (in place; returns the job)."""
    for st in job.stations:
        if not isinstance(st.frames, torch.Tensor):
            st.frames = torch.from_numpy(np.ascontiguousarray(st.frames).view(np.int32))
        st.frames = st.frames.to(device).contiguous()
    return job


class XcServerStats(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("completed", C.c_int64), ("failed", C.c_int64), ("cancelled", C.c_int64),
                ("queued", C.c_int64), ("running", C.c_int64),
                ("station_samples_per_s", C.c_double)]


def _server_sigs(lib):
    P = C.c_void_p
    sig = {
        "xc_server_create": (C.c_int, [C.POINTER(P), C.c_int, C.c_size_t, C.c_int32]),
        "xc_server_submit": (C.c_int, [P, C.POINTER(XcJob), C.POINTER(C.c_uint64)]),
        "xc_server_poll": (C.c_int, [P, C.c_uint64, C.POINTER(C.c_int32)]),
        "xc_server_wait": (C.c_int, [P, C.c_uint64, C.c_int32]),
        "xc_server_cancel": (C.c_int, [P, C.c_uint64]),
        "xc_server_get_stats": (C.c_int, [P, C.POINTER(XcServerStats)]),
        "xc_server_last_error": (C.c_char_p, [P]),
        "xc_server_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


class Server:
    """Continuous-batching server (xc_server_*): submit jobs, poll/wait, stats."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 16 << 30, max_slots: int = 4):
        self.lib = load_library()
        _server_sigs(self.lib)
        self.device = device
        self.srv = C.c_void_p()
        rc = self.lib.xc_server_create(C.byref(self.srv), device, hbm_budget_bytes, max_slots)
        if rc != XC_OK:
            raise XcError(rc, strerror(rc))
        self._keep = {}

    def _check(self, rc):
        if rc != XC_OK:
            raise XcError(rc, f"{strerror(rc)}: {self.lib.xc_server_last_error(self.srv).decode()}")

    def submit(self, job, *, precision: int = XC_FP32, out=None):
        """Queue a job; returns (ticket, (vis, weight)).  Outputs fill when it is done."""
        m = _Marshal(job, precision)
        if out is None:
            dev = f"cuda:{self.device}"
            out = (torch.empty(job.n_subbands, job.n_baselines, job.n_chan, dtype=torch.complex64,
                               device=dev),
                   torch.empty(job.n_subbands, job.n_baselines, dtype=torch.float32, device=dev))
        torch.cuda.current_stream(self.device).synchronize()   # recordings and outputs are ready
        arr = XcJob(m.setup, C.cast(m.stations, C.POINTER(XcStation)),
                    XcOutput(out[0].data_ptr(), out[1].data_ptr()))
        t = C.c_uint64()
        self._check(self.lib.xc_server_submit(self.srv, C.byref(arr), C.byref(t)))
        self._keep[t.value] = (job, out)
        return t.value, out

    def poll(self, ticket: int):
        d = C.c_int32()
        rc = self.lib.xc_server_poll(self.srv, ticket, C.byref(d))
        return bool(d.value), rc

    def wait(self, ticket: int, timeout_ms: int = -1) -> int:
        rc = self.lib.xc_server_wait(self.srv, ticket, timeout_ms)
        if rc != XC_E_TIMEOUT:
            self._keep.pop(ticket, None)
        return rc

    def cancel(self, ticket: int) -> int:
        return self.lib.xc_server_cancel(self.srv, ticket)

    def stats(self) -> dict:
        s = XcServerStats()
        self._check(self.lib.xc_server_get_stats(self.srv, C.byref(s)))
        return {f: getattr(s, f) for f, _ in XcServerStats._fields_}

    def close(self):
        if self.srv:
            self.lib.xc_server_destroy(self.srv)
            self.srv = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
