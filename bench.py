"""Throughput benchmark of the FX correlation path on one MI355X.

One step = one whole sub-integration through the C ABI (A0 ingest .. A8
finalise) on inputs already resident in HBM.  Default workload: 10 stations
(1 space + 9 ground), 8 x 16 MHz subbands, dual pol (16 recorded streams),
1024 channels, 4 s = 62 500 FFT frames of 2048 samples per input.

Prints one JSON line (stdout).  Progress goes to stderr.

  python bench.py [--steps K] [--warmup W] [--workload c2|c1|c4] [--no-cpu-baseline]
  python bench.py --workload c4 --precision fp16|fp8|fp32   # X stage on MFMA (FP16/FP8) or FP32
  python bench.py --workload c3        # 64 uneven jobs: batch (lanes + hipGraph) vs per-job loop
  python bench.py --workload c3 --job-mix short --no-autotune   # 256 short jobs, the same comparison
  python bench.py --workload c5        # Poisson request trace through the server
  python bench.py --workload fringe    # delay-rate fringe search over a C2-shaped scan
  python bench.py --workload feed      # feed-angle correction over a C2-shaped scan
  python bench.py --workload xcross    # X stage: vector and matrix-core FP32, MFMA FP16 / e4m3 as inputs grow
  python bench.py --workload fstage-n  # F and X stage throughput by FFT length (single-pol jobs)
  python bench.py --calibrate-copy     # plain device copy of known size, for counter scaling
  python bench.py --rocpd-summary DB   # per-kernel table from a rocprofv3 database
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3       # MI355X vector FP32, published (counts packed FP32 FMA)
# The issue ceiling of this build's FP32 code: packed-FP32 instructions are
# disabled, so one FMA per lane per cycle: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops x 2.4 GHz.  Reported beside the published peak, never in its place.
FP32_ISSUE_CEILING_TFS = 78.6


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1502_06894_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


F_SOURCES = ["k_fstage.hip", "xc_fft.h", "xc_dev.h"]
X_SOURCES = ["k_xmac.hip", "xc_dev.h"]


def make_job(name: str, frames: int = 0):
    from synth import configs
    if name == "c2":
        kw = {"n_frames": frames} if frames else {}
        return configs.c2_job(device="cuda", realistic=True, **kw), (
            "C2: 10 stations (1 space + 9 ground), 8 x 16 MHz subbands, dual pol, "
            "1024 channels, 4 s sub-int, 2-bit")
    if name == "c1":
        return configs.c1_job(device="cuda"), ("C1: 2 stations (space + ground), 1 x 16 MHz, single pol, "
                                  "256 channels, 0.5 s, 2-bit, exact-physics generator")
    if name == "c4":
        return configs.c4_job(device="cuda"), (
            "C4: 32 stations, 4 x 32 MHz subbands, single pol, 4096 channels, 1 s, 2-bit")
    raise SystemExit(f"unknown workload {name}")


def traffic_from_profile(kind: str, src_hash: str):
    """HBM bytes per station-sample of a kernel kind, from the counter summary
    profiles/hbm_counters.json (FETCH_SIZE + WRITE_SIZE, scaled by a plain
    copy's counts), or None when it is missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", "hbm_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    e = d.get(kind)
    if not e or e.get("source_hash") != src_hash:
        return None
    return e.get("bytes_per_station_sample")


# Vector-instruction issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions/s
# (a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles).
VALU_ISSUE_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def valu_from_profile(kind: str, src_hash: str):
    """VALU instructions per station-sample and VALU busy of a kernel kind from
    profiles/valu_counters.json (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU), or None."""
    path = os.path.join(ROOT, "profiles", "valu_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        e = json.load(fh).get(kind)
    if not e or e.get("source_hash") != src_hash:
        return None
    return e


def roofline(kind: str, bytes_per_ss: float, flops_per_ss: float, src_files, prof_entry,
             ss_total: float) -> dict:
    """Roofline record of one kernel kind from its live HIP-event time.

    T_bound = max(bytes / 8 TB/s, flops / 157.3 TFLOP/s) per launch (published
    MI355X peaks); the roof with the larger time binds; frac = T_bound / T_meas.
    `traffic` is the HBM bytes per launch measured by the FETCH_SIZE and
    WRITE_SIZE counters (committed summary, same kernel sources) or null."""
    ms_tot, n_launch = prof_entry
    t_meas = ms_tot * 1e-3 / n_launch
    ss_launch = ss_total / n_launch
    alg_bytes = bytes_per_ss * ss_launch
    alg_flops = flops_per_ss * ss_launch
    t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
    t_alu = alg_flops / (FP32_PEAK_TFLOPS * 1e12)
    src_hash = kernel_source_hash(src_files)
    tr = traffic_from_profile(kind, src_hash)
    hbm = {"achieved": round(alg_bytes / t_meas / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(t_hbm / t_meas, 4)}
    alu = {"achieved": round(alg_flops / t_meas / 1e12, 2), "peak": FP32_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(t_alu / t_meas, 4),
           "issue_ceiling_nonpacked_tflops": FP32_ISSUE_CEILING_TFS,
           "frac_of_issue_ceiling": round(alg_flops / t_meas / 1e12 / FP32_ISSUE_CEILING_TFS, 4)}
    bound = "hbm" if t_hbm >= t_alu else "alu"
    main, side = (hbm, alu) if bound == "hbm" else (alu, hbm)
    v = valu_from_profile(kind, src_hash)
    valu = None
    if v is not None:
        rate = v["instr_per_station_sample"] * ss_launch / t_meas / 1e12
        valu = {"instr_per_station_sample": round(v["instr_per_station_sample"], 2),
                "achieved_tera_lane_instr_per_s": round(rate, 2),
                "peak_at_2p4_ghz": round(VALU_ISSUE_PEAK_T, 2),
                "frac": round(rate / VALU_ISSUE_PEAK_T, 4),
                "valu_busy_counter": round(v["valu_busy"], 3)}
        if "mfma_busy" in v:
            valu["mfma_busy_counter"] = round(v["mfma_busy"], 3)
    return {"bound": bound, "achieved": main["achieved"], "peak": main["peak"],
            "unit": main["unit"], "frac": main["frac"],
            "traffic": None if tr is None else round(tr * ss_launch),
            "kernel": kind, "kernel_ms_per_launch": round(t_meas * 1e3, 4),
            "launches": n_launch,
            "algorithmic_bytes_per_launch": round(alg_bytes),
            "algorithmic_flops_per_launch": round(alg_flops),
            "bytes_per_station_sample": bytes_per_ss, "flops_per_station_sample": flops_per_ss,
            "arithmetic_intensity_flop_per_byte": round(flops_per_ss / bytes_per_ss, 2),
            "ridge_flop_per_byte": round(FP32_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS, 2),
            "source_hash": src_hash,
            ("alu" if bound == "hbm" else "hbm"): side,
            "valu_issue": valu}


def cpu_model() -> str:
    """The host CPU's model name (Linux), for the CPU-baseline record."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(job, budget_s: float = 12.0, max_frames: int = 8192):
    """The FP64 oracle on a bounded sample of the same workload (subband 0, all inputs)."""
    import torch
    from oracle import fx
    from synth.job import Job, Station

    cores = min(16, os.cpu_count() or 1)
    spf = 40000 // job.n_streams
    stations = []
    for st in job.stations:
        n_int, _ = fx.frame_delays(st.delay_poly, job.sub_start, job.N, job.fs_hz,
                                   np.array([0, max_frames - 1]))
        base = job.sub_start + np.array([0, max_frames - 1]) * job.N + n_int - st.first_sample
        lo = max(0, int(base.min()) // spf - 1)
        hi = min(st.n_frames_m5b, (int(base.max()) + job.N) // spf + 2)
        stations.append(Station(frames=st.frames[lo:hi].cpu(), first_sample=st.first_sample + lo * spf,
                                delay_poly=st.delay_poly, phase_poly=st.phase_poly,
                                poly_span=st.poly_span, station_id=st.station_id,
                                rate_correct=st.rate_correct))
    sub = Job(n_stations=job.n_stations, n_subbands=job.n_subbands, n_pols=job.n_pols,
              n_chan=job.n_chan, n_streams=job.n_streams, stream_map=job.stream_map,
              fs_hz=job.fs_hz, lo_hz=job.lo_hz, sub_start=job.sub_start, n_frames=max_frames,
              stations=stations)
    chunk = 64 * cores            # one call spreads 64-frame chunks over all threads
    done = 0
    t0 = time.perf_counter()
    while done < max_frames and time.perf_counter() - t0 < budget_s:
        n = min(chunk, max_frames - done)
        fx.correlate(sub, subbands=[0], frames=np.arange(done, done + n), threads=cores, chunk=64)
        done += n
    dt = time.perf_counter() - t0
    ss = job.M * done * job.N
    return {"value": ss / dt / 1e9, "unit": "G station-samples/s", "cores": cores,
            "cpu": cpu_model(), "kind": "oracle",
            "sample": f"subband 0 of {job.n_subbands}, all {job.M} inputs, frames 0..{done - 1} "
                      f"of {job.n_frames} ({ss:.3e} station-samples in {dt:.1f} s, "
                      f"{cores} threads)"}


def short_kernel_name(name: str) -> str:
    """'void xc::k_fstage<2048>(...)' -> 'xc::k_fstage<2048>'; other names cut to 60 chars."""
    n = name.replace("void ", "", 1).replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:i]
            break
    return n[:60]


def rocpd_summary(db_path: str) -> str:
    """Per-kernel dispatch statistics (and counter means) from a rocprofv3 rocpd database."""
    import sqlite3
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    lines = []
    rows = cur.execute("select name, duration, lds_size, scratch_size, vgpr_count, "
                       "accum_vgpr_count, grid_x, grid_y, grid_z, workgroup_x from kernels")
    stats = {}
    for name, dur, lds, scr, vgpr, agpr, gx, gy, gz, wx in rows:
        k = short_kernel_name(name)
        e = stats.setdefault(k, {"n": 0, "tot": 0.0, "min": 1e30, "max": 0.0,
                                 "res": (vgpr, agpr, lds, scr, wx)})
        e["n"] += 1
        e["tot"] += dur
        e["min"] = min(e["min"], dur)
        e["max"] = max(e["max"], dur)
    if stats:
        lines.append(f"{'kernel':60s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s} "
                     f"{'min_us':>9s} {'max_us':>9s}  vgpr agpr lds scratch wg")
        for k, e in sorted(stats.items(), key=lambda kv: -kv[1]["tot"]):
            v, a, l, sc, wx = e["res"]
            lines.append(f"{k:60s} {e['n']:6d} {e['tot'] / 1e6:10.3f} {e['tot'] / e['n'] / 1e3:10.2f} "
                         f"{e['min'] / 1e3:9.2f} {e['max'] / 1e3:9.2f}  {v} {a} {l} {sc} {wx}")
    try:
        rows = list(cur.execute("select kernel_name, counter_name, value from counters_collection"))
    except sqlite3.OperationalError:
        rows = []
    if rows:
        agg = {}
        for kn, cn, val in rows:
            e = agg.setdefault((short_kernel_name(kn), cn), [0, 0.0])
            e[0] += 1
            e[1] += val
        lines.append("")
        lines.append(f"{'kernel':60s} {'counter':16s} {'dispatches':>10s} {'mean/dispatch':>16s}")
        for (k, cn), (n, tot) in sorted(agg.items()):
            lines.append(f"{k:60s} {cn:16s} {n:10d} {tot / n:16.1f}")
    return "\n".join(lines)


def _counter_means(db_path: str, counter: str) -> dict:
    """Mean value per dispatch of one counter, per short kernel name (rocpd database)."""
    import sqlite3
    cur = sqlite3.connect(db_path).cursor()
    agg = {}
    for kn, cn, val in cur.execute("select kernel_name, counter_name, value "
                                   "from counters_collection"):
        if cn != counter:
            continue
        e = agg.setdefault(short_kernel_name(kn), [0, 0.0])
        e[0] += 1
        e[1] += val
    return {k: tot / n for k, (n, tot) in agg.items()}


# The C2 workload's F and X kernels in a counter database: the F-stage and
# X-stage kernels of its FFT length and input count, whatever variant the
# library's defaults pick (the one with the most dispatches).
C2_KERNELS = {"fstage": (("xc::k_fstage<2048,",), F_SOURCES),
              "xmac": (("xc::k_xmac_ringm<20,", "xc::k_xmac_ring<20,", "xc::k_xmac_mfma<5,"),
                       X_SOURCES)}


def _resolve_kernels(counts: dict, kernels: dict) -> dict:
    out = {}
    for kind, (prefixes, srcs) in kernels.items():
        names = [n for n in counts if n.startswith(prefixes)]
        if not names:
            raise SystemExit(f"no kernel {' / '.join(prefixes)}... in the counter database")
        out[kind] = (max(names, key=lambda n: counts[n]), srcs)
    return out


def _dispatch_counts(db_path: str, counter: str) -> dict:
    import sqlite3
    cur = sqlite3.connect(db_path).cursor()
    n = {}
    for kn, cn in cur.execute("select kernel_name, counter_name from counters_collection"):
        if cn == counter:
            k = short_kernel_name(kn)
            n[k] = n.get(k, 0) + 1
    return n


def valu_json(db: str, ss_per_launch: float, kernels: dict) -> dict:
    """VALU instructions per station-sample (SQ_INSTS_VALU x 64 / ss), VALU
    busy (SQ_ACTIVE_INST_VALU / (256 CUs x GRBM_GUI_ACTIVE / 8 XCDs)) and, where
    the run also counted SQ_VALU_MFMA_BUSY_CYCLES, matrix-core busy per kernel kind."""
    insts = _counter_means(db, "SQ_INSTS_VALU")
    active = _counter_means(db, "SQ_ACTIVE_INST_VALU")
    grbm = _counter_means(db, "GRBM_GUI_ACTIVE")
    mfma = _counter_means(db, "SQ_VALU_MFMA_BUSY_CYCLES")
    kernels = _resolve_kernels(_dispatch_counts(db, "SQ_INSTS_VALU"), kernels)
    out = {"ss_per_launch": ss_per_launch}
    for kind, (name, srcs) in kernels.items():
        out[kind] = {"kernel": name, "source_hash": kernel_source_hash(srcs),
                     "instr_per_station_sample": insts[name] * 64.0 / ss_per_launch,
                     "valu_busy": active[name] / (256.0 * grbm[name] / 8.0)}
        if name in mfma:
            # matrix-core busy cycles over 1024 SIMDs x the cycles of one XCD
            out[kind]["mfma_busy"] = mfma[name] / (1024.0 * grbm[name] / 8.0)
    return out


def traffic_json(fetch_db: str, write_db: str, copy_fetch_db: str, copy_write_db: str,
                 ss_per_launch: float, kernels: dict) -> dict:
    """HBM bytes per station-sample of each kernel kind from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the counter reads for a
    plain 1 GiB device copy (which reads and writes 1 GiB)."""
    copy_kib = (1 << 30) / 1024.0
    cf = _counter_means(copy_fetch_db, "FETCH_SIZE")["__amd_rocclr_copyBuffer"]
    cw = _counter_means(copy_write_db, "WRITE_SIZE")["__amd_rocclr_copyBuffer"]
    sf, sw = copy_kib / cf, copy_kib / cw
    fetch = _counter_means(fetch_db, "FETCH_SIZE")
    write = _counter_means(write_db, "WRITE_SIZE")
    kernels = _resolve_kernels(_dispatch_counts(fetch_db, "FETCH_SIZE"), kernels)
    out = {"fetch_scale": sf, "write_scale": sw, "ss_per_launch": ss_per_launch}
    for kind, (name, srcs) in kernels.items():
        fb = fetch[name] * sf * 1024.0
        wb = write[name] * sw * 1024.0
        out[kind] = {"kernel": name, "source_hash": kernel_source_hash(srcs),
                     "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
                     "bytes_per_station_sample": (fb + wb) / ss_per_launch}
    return out


def calibrate_read():
    """Read ceiling: a 4 GiB float32 sum (torch's reduction, HIP events)."""
    import torch
    x = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    for _ in range(3):
        x.sum()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        x.sum()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    print(json.dumps({"read_bytes": 4 << 30, "ms": round(ms, 4),
                      "gb_per_s": round((4 << 30) / (ms * 1e-3) / 1e9, 1)}))


def calibrate_copy():
    import torch
    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "dispatches": 5}))


def _default_fpb(job, elem_bytes=8):
    """The library's default frames per block: 2048, or up to 65536 while the
    block's staged spectra stay within 16 GiB."""
    per_frame = job.n_subbands * job.M * job.n_chan * elem_bytes
    return int(min(max(2048, min(65536, (16 << 30) // per_frame)), job.n_frames))


def _batch_fpb(job, tuned_fpb=0, elem_bytes=8):
    """Frames per block a batch gives a job: the tuned size (else the library
    default), capped as for every job sharing the device (1 GiB, at least 64),
    except that a job the cap would cut into more than 4 blocks keeps the
    uncapped size (it runs alone on the batch's first lane)."""
    T = min(tuned_fpb, job.n_frames) if tuned_fpb else _default_fpb(job, elem_bytes)
    t = _shared_fpb(job, T, 1 << 30, 64, elem_bytes)
    if t != T and -(-job.n_frames // t) > 4:
        return int(T)
    return t


# X-stage staging values of the library's tuning record, by name
XSTAGING = {0: "default", 1: "direct", 2: "2-frame stages", 3: "matrix cores",
            4: "4-frame stages", 5: "matrix cores through the ring", 8: "ring"}


def run_c3(a):
    """64 uneven sub-integrations over a device-resident pool: the fused batch
    executor (one persistent F-stage launch per FFT length and round) and the
    lane executor against the per-job loop, with tile shapes from the autotuner."""
    import torch
    from paper_1502_06894_amd import xcorr
    from synth import configs
    log("generating the 20-station x 16-stream x 4.5 s pool on the GPU")
    pool = configs.pool_recordings(device="cuda")
    short = a.job_mix == "short"
    jobs = (configs.short_batch_jobs(pool, a.jobs or 256) if short
            else configs.batch_jobs(pool, a.jobs or 64))
    torch.cuda.synchronize()
    ss = sum(j.station_samples for j in jobs)
    log(f"{len(jobs)} jobs, {ss:.3e} station-samples")
    corr = xcorr.Correlator(0)
    tuned = [{} for _ in jobs]
    if not a.no_autotune:
        # candidates that need more than 8 GiB of workspace are skipped
        wst = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
        t0 = time.perf_counter()
        for k, j in enumerate(jobs):
            tuned[k] = corr.autotune(j, workspace=wst)
            if (k + 1) % 8 == 0:
                log(f"  autotuned {k + 1} jobs ({time.perf_counter() - t0:.1f} s)")
        del wst
        torch.cuda.synchronize()
    picks = {}
    for t in tuned:
        xs = t.get("xmac_frames_per_stage", 0)
        key = (f"fpb {t.get('frames_per_block', 0)}, X stage {XSTAGING.get(xs, f'staging {xs}')}"
               + (f" {t['xmac_channels_per_wg']} ch" if t.get("xmac_channels_per_wg") else ""))
        picks[key] = picks.get(key, 0) + 1
    fpbs = [_batch_fpb(j, t.get("frames_per_block", 0)) for j, t in zip(jobs, tuned)]
    # per-job loop at the batch's block sizes
    outs = [corr.alloc_output(j) for j in jobs]
    ws = torch.empty(max(corr.workspace_bytes(j, frames_per_block=f) for j, f in zip(jobs, fpbs)),
                     dtype=torch.uint8, device="cuda")

    def loop():
        for j, f, o in zip(jobs, fpbs, outs):
            corr.correlate(j, frames_per_block=f, out=o, workspace=ws)

    loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        loop()
    torch.cuda.synchronize()
    t_loop = (time.perf_counter() - t0) / a.steps
    log(f"per-job loop: {t_loop * 1e3:.1f} ms per batch, {ss / t_loop / 1e9:.1f} G ss/s")
    refs = [(v.clone(), w.clone()) for v, w in outs]
    del ws
    # the plain per-job path a caller gets without choosing block sizes: the
    # library's default blocks (up to 16 GiB of spectra; the tuned size where
    # the autotuner picked one)
    dfl = [t.get("frames_per_block", 0) for t in tuned]
    ws = torch.empty(max(corr.workspace_bytes(j, frames_per_block=f) for j, f in zip(jobs, dfl)),
                     dtype=torch.uint8, device="cuda")
    for j, f, o in zip(jobs, dfl, outs):
        corr.correlate(j, frames_per_block=f, out=o, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        for j, f, o in zip(jobs, dfl, outs):
            corr.correlate(j, frames_per_block=f, out=o, workspace=ws)
    torch.cuda.synchronize()
    t_dfl = (time.perf_counter() - t0) / a.steps
    log(f"per-job loop at the library's default blocks: {t_dfl * 1e3:.1f} ms per batch, "
        f"{ss / t_dfl / 1e9:.1f} G ss/s")
    del ws
    lanes = a.lanes or 8
    res = {}
    for name, lanes_only in (("lanes", True), ("fused", False)):
        bws = corr.batch_workspace(jobs, n_lanes=lanes, lanes_only=lanes_only)
        bouts = [corr.alloc_output(j) for j in jobs]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            corr.correlate_batch(jobs, n_lanes=lanes, graph=True, lanes_only=lanes_only,
                                 outs=bouts, workspace=bws, stream=stream)     # capture
            stream.synchronize()
            corr.profile_begin(200000)
            t0 = time.perf_counter()
            for _ in range(a.steps):
                corr.correlate_batch(jobs, n_lanes=lanes, graph=True, lanes_only=lanes_only,
                                     outs=bouts, workspace=bws, stream=stream)
            stream.synchronize()
            tb = (time.perf_counter() - t0) / a.steps
            prof = corr.profile_end()
        same = all(torch.equal(v, rv) and torch.equal(w, rw)
                   for (v, w), (rv, rw) in zip(bouts, refs))
        res[name] = {"value": round(ss / tb / 1e9, 2), "ms_per_step": round(tb * 1e3, 3),
                     "over_per_job_loop": round(t_loop / tb, 3),
                     "over_per_job_default_blocks": round(t_dfl / tb, 3),
                     "identical_to_per_job": bool(same),
                     "workspace_gb": round(bws.numel() / 1e9, 2)}
        log(f"batch {name} ({lanes} lanes, graph replay): {tb * 1e3:.1f} ms, "
            f"{ss / tb / 1e9:.1f} G ss/s ({t_loop / tb:.3f}x the per-job loop, "
            f"{t_dfl / tb:.3f}x at default blocks); identical: {same}")
        del bws, bouts
        torch.cuda.synchronize()
    f = res["fused"]
    return {
        "metric": "correlated station-samples/s", "value": f["value"],
        "unit": "G station-samples/s", "n_gpus": 1, "steps": a.steps, "warmup": 1,
        "ms_per_step": f["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{len(jobs)} short sub-integration jobs (stations 2-6, subbands "
                                f"1-4, channels 128-1024, 0.01-0.1 s) over a 20-station x "
                                f"16-stream x 4.5 s device-resident pool" if short else
                                f"C3: {len(jobs)} uneven sub-integration jobs (stations 2-20, "
                                f"subbands 1-16, channels 128-8192, 0.1-4 s) over a 20-station "
                                f"x 16-stream x 4.5 s device-resident pool"),
                   "lanes": lanes, "graph": True, "station_samples_per_step": ss,
                   "autotuned": not a.no_autotune},
        "per_job_loop": {"value": round(ss / t_loop / 1e9, 2), "ms_per_step": round(t_loop * 1e3, 3),
                         "blocks": "the batch's"},
        "per_job_loop_default_blocks": {"value": round(ss / t_dfl / 1e9, 2),
                                        "ms_per_step": round(t_dfl * 1e3, 3)},
        "fused": f, "lanes": res["lanes"],
        "batch_over_loop": f["over_per_job_loop"],
        "identical_to_per_job": f["identical_to_per_job"] and res["lanes"]["identical_to_per_job"],
        "autotune_picks": picks,
    }


def _correlator(a):
    """A library context with the --tune overrides (none: the library defaults)."""
    from paper_1502_06894_amd import xcorr
    corr = xcorr.Correlator(0)
    if a.tune:
        corr.set_tuning(**{k: int(v) for k, v in (kv.split("=", 1) for kv in a.tune)})
        log(f"tuning: {corr.get_tuning()}")
    return corr


def run_c4(a):
    """32 stations, 4 x 32 MHz, 4096 channels, 1 s, FP32 / FP16 / FP8 X stage."""
    import torch
    from paper_1502_06894_amd import xcorr
    job, desc = make_job("c4")
    xcorr.job_to_device(job, "cuda:0")
    corr = _correlator(a)
    res = {}
    for prec in ("fp32", "fp16", "fp8"):
        p = xcorr.PRECISIONS[prec]
        ws = corr.alloc_workspace(job, precision=p)
        out = corr.alloc_output(job)
        for _ in range(a.warmup):
            corr.correlate(job, precision=p, out=out, workspace=ws)
        torch.cuda.synchronize()
        # timed without the library's per-launch events (two HIP event records
        # around each of the ~50 launches of a step perturb the short ones
        # here); the kernel breakdown comes from a second, profiled pass
        t0 = time.perf_counter()
        for _ in range(a.steps):
            corr.correlate(job, precision=p, out=out, workspace=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        corr.profile_begin(a.steps * 128 + 64)
        t1 = time.perf_counter()
        for _ in range(a.steps):
            corr.correlate(job, precision=p, out=out, workspace=ws)
        torch.cuda.synchronize()
        dt_prof = (time.perf_counter() - t1) / a.steps
        prof = corr.profile_end()
        res[prec] = {"value": round(job.station_samples / dt / 1e9, 2), "ms_per_step": round(dt * 1e3, 3),
                     "profiled_ms_per_step": round(dt_prof * 1e3, 3),
                     "kernels_ms_per_step": {k: round(ms / a.steps, 3) for k, (ms, n) in prof.items() if n}}
        log(f"C4 {prec}: {dt * 1e3:.2f} ms/step, {job.station_samples / dt / 1e9:.1f} G ss/s "
            f"{res[prec]['kernels_ms_per_step']}")
        del ws
    main_p = a.precision
    return {
        "metric": "correlated station-samples/s", "value": res[main_p]["value"],
        "unit": "G station-samples/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": res[main_p]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "fp16": "f16 in, f32 accumulate",
                                       "fp8": "e4m3 in, f32 accumulate"}[main_p],
        "data": "synthetic",
        "config": {"workload": desc, "stations": job.n_stations, "subbands": job.n_subbands,
                   "channels": job.n_chan, "frames": job.n_frames, "precision": main_p,
                   "station_samples_per_step": job.station_samples},
        "precisions": res,
    }


def _shared_fpb(job, T, cap, min_frames, elem_bytes=8):
    """The library's block size for a job sharing the device (a batch, a served
    request): T, with the staged spectra capped at `cap` bytes but never fewer
    than 16 (M + 1) frames (its FP64 accumulator traffic per block) nor
    min_frames."""
    per_frame = job.n_subbands * job.M * job.n_chan * elem_bytes
    if T * per_frame <= cap:
        return int(T)
    t = max(cap // per_frame, min(T, 16 * (job.M + 1)), min_frames)
    return int(min(t, T))


def _server_fpb(job, budget, slots, elem_bytes=8):
    """Frames per block the server gives a request: its spectra capped at half
    the budget shared among the slots (at least 1 GiB), at least 16 frames."""
    cap = max(1 << 30, budget // (2 * slots))
    return _shared_fpb(job, _default_fpb(job, elem_bytes), cap, 16, elem_bytes)


def run_c5(a):
    """Poisson request trace through the continuous-batching server, against
    the same requests run one after another through the plain per-job path;
    a sample of the served results is checked bit for bit against the same
    request run alone."""
    import torch
    from paper_1502_06894_amd import xcorr
    from synth import configs
    log("generating the 20-station x 16-stream x 4.5 s pool on the GPU")
    pool = configs.pool_recordings(device="cuda")
    trace = configs.serve_trace(pool, a.requests, rate_hz=a.rate, max_log2_chan=a.max_log2_chan)
    jobs = [j for _, j in trace]
    ss = sum(j.station_samples for j in jobs)
    span = trace[-1][0]
    # outputs allocated up front, so that no allocation runs beside the server
    outs = [(torch.empty(j.n_subbands, j.n_baselines, j.n_chan, dtype=torch.complex64,
                         device="cuda"),
             torch.empty(j.n_subbands, j.n_baselines, dtype=torch.float32, device="cuda"))
            for j in jobs]
    torch.cuda.synchronize()
    log(f"{len(trace)} requests over {span:.2f} s, offered {ss / span / 1e9:.1f} G ss/s, "
        f"outputs {sum(v.numel() * 8 for v, _ in outs) / 1e9:.1f} GB")
    slots = a.lanes or 16      # more slots than C3's lanes: small requests need not queue
    srv = xcorr.Server(0, hbm_budget_bytes=a.budget_gb << 30, max_slots=slots)
    tickets = []
    t0 = time.perf_counter()
    for (arr, job), o in zip(trace, outs):
        now = time.perf_counter() - t0
        if arr > now:
            time.sleep(arr - now)
        tickets.append(srv.submit(job, out=o)[0])
    rcs = []
    for k, t in enumerate(tickets):
        rcs.append(srv.wait(t))
        if (k + 1) % 250 == 0:
            log(f"  {k + 1} requests served")
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    log(f"served {st['completed']} requests in {wall:.2f} s: p50 {st['p50_ms']:.1f} ms, "
        f"p99 {st['p99_ms']:.1f} ms, {st['station_samples_per_s'] / 1e9:.1f} G ss/s")

    # the same requests through the plain per-job path, one after another
    # (library defaults, one workspace sized for the largest request)
    corr = xcorr.Correlator(0)
    ws = torch.empty(max(corr.workspace_bytes(j) for j in jobs), dtype=torch.uint8, device="cuda")
    o1 = (torch.empty(max(v.numel() for v, _ in outs), dtype=torch.complex64, device="cuda"),
          torch.empty(max(w.numel() for _, w in outs), dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k, j in enumerate(jobs):
        v = o1[0][:j.n_subbands * j.n_baselines * j.n_chan].view(j.n_subbands, j.n_baselines,
                                                                  j.n_chan)
        w = o1[1][:j.n_subbands * j.n_baselines].view(j.n_subbands, j.n_baselines)
        corr.correlate(j, out=(v, w), workspace=ws)
        if (k + 1) % 250 == 0:
            torch.cuda.synchronize()
            log(f"  per-job path: {k + 1} requests")
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t1
    loop_gss = ss / t_loop / 1e9
    log(f"per-job path: {t_loop:.2f} s, {loop_gss:.1f} G ss/s")

    # alone vs in the mix: every k-th served request run alone with the
    # server's block size must give the same bits
    n_check = min(a.check_jobs, len(jobs))
    idx = np.linspace(0, len(jobs) - 1, n_check).round().astype(int).tolist()
    same = 0
    for i in idx:
        j = jobs[i]
        v, w = corr.correlate(j, frames_per_block=_server_fpb(j, a.budget_gb << 30, slots))
        same += int(torch.equal(v, outs[i][0]) and torch.equal(w, outs[i][1]))
    torch.cuda.synchronize()
    log(f"alone == in the mix, bit for bit: {same} of {n_check} sampled requests")
    served = st["station_samples_per_s"] / 1e9
    return {
        "metric": "correlated station-samples/s", "value": round(served, 2),
        "unit": "G station-samples/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(wall * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"C5: Poisson trace, {len(trace)} requests at {a.rate:g}/s "
                               f"(stations 3-20, subbands 1-16, channels 256-{2 ** a.max_log2_chan}, "
                               f"0.1-4 s) over the device-resident pool",
                   "slots": slots, "hbm_budget_gb": a.budget_gb,
                   "station_samples": ss},
        "latency_ms": {"p50": round(st["p50_ms"], 2), "p99": round(st["p99_ms"], 2),
                       "mean": round(st["mean_ms"], 2)},
        "offered_g_per_s": round(ss / span / 1e9, 2),
        "per_job_path": {"value": round(loop_gss, 2), "seconds": round(t_loop, 3)},
        "served_over_per_job": round(served / loop_gss, 3),
        "alone_equals_mix": {"checked": n_check, "identical": same},
        "completed": st["completed"], "failed": st["failed"],
        "all_ok": all(rc == 0 for rc in rcs),
    }


def run_xcross(a):
    """X stage on the vector ALUs (FP32), on the matrix cores in FP32 (the same
    fused multiply-adds, bit-identical sums; operands loaded per wave or fed
    through the LDS ring) and on MFMA in FP16 / e4m3, as the
    number of inputs per subband grows: C4-shaped jobs (4 x 32 MHz subbands,
    4096 channels, 1024 frames) with M = 4 .. 32 stations, X-stage kernel time
    per job from HIP events."""
    import torch
    from paper_1502_06894_amd import xcorr
    from synth import configs
    corr = xcorr.Correlator(0)
    rows = []
    # (name, precision, X staging): FP32 on the vector ALUs through the LDS
    # ring, FP32 on the matrix cores, FP16 / e4m3 on MFMA
    variants = (("fp32", "fp32", 8), ("fp32m", "fp32", xcorr.XMAC_MATRIX),
                ("fp32mr", "fp32", xcorr.XMAC_MATRIX_RING), ("fp16", "fp16", 0), ("fp8", "fp8", 0))
    for M in (4, 8, 12, 16, 20, 24, 28, 32):
        job = configs.c4_job(device="cuda", n_stations=M, n_frames=1024)
        xcorr.job_to_device(job, "cuda:0")
        row = {"inputs": M}
        vis32 = {}
        for name, prec, xs in variants:
            p = xcorr.PRECISIONS[prec]
            corr.set_tuning(xmac_frames_per_stage=xs)
            ws = corr.alloc_workspace(job, precision=p)
            out = corr.alloc_output(job)
            for _ in range(a.warmup):
                corr.correlate(job, precision=p, out=out, workspace=ws)
            torch.cuda.synchronize()
            corr.profile_begin(a.steps * 64 + 64)
            for _ in range(a.steps):
                corr.correlate(job, precision=p, out=out, workspace=ws)
            torch.cuda.synchronize()
            prof = corr.profile_end()
            kind = "xmfma" if prec != "fp32" else "xmac"
            ms = prof[kind][0] / a.steps
            eb = {"fp32": 8, "fp16": 4, "fp8": 2}[prec]
            gb = job.n_subbands * job.n_frames * job.M * job.n_chan * eb / 1e9
            row[name] = {"x_ms": round(ms, 4), "spectra_gb_per_s": round(gb / (ms * 1e-3), 1),
                         "f_ms": round(prof["fstage"][0] / a.steps, 4)}
            if prec == "fp32":
                vis32[name] = out[0].clone()
            del ws, out
        corr.set_tuning(xmac_frames_per_stage=0)
        row["fp32m_bit_identical"] = bool(torch.equal(vis32["fp32"], vis32["fp32m"]))
        row["fp32mr_bit_identical"] = bool(torch.equal(vis32["fp32"], vis32["fp32mr"]))
        rows.append(row)
        log(f"M = {M:2d}: X stage FP32 vector {row['fp32']['x_ms']:.3f} ms, matrix "
            f"{row['fp32m']['x_ms']:.3f} ms (identical: {row['fp32m_bit_identical']}), "
            f"matrix through the ring {row['fp32mr']['x_ms']:.3f} ms (identical: "
            f"{row['fp32mr_bit_identical']}), "
            f"FP16 {row['fp16']['x_ms']:.3f} ms, e4m3 {row['fp8']['x_ms']:.3f} ms")
        del job, vis32
        torch.cuda.synchronize()
    return {"metric": "X-stage time per job (ms), vector FP32 vs matrix-core FP32 vs MFMA "
                      "FP16/e4m3", "value": None,
            "unit": "ms", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "higher_is_better": False, "data": "synthetic",
            "config": {"workload": "C4-shaped jobs: 4 x 32 MHz subbands, 4096 channels, "
                                   "1024 frames, M = 4..32 single-pol stations"},
            "rows": rows}


def run_fstage_n(a):
    """F- and X-stage throughput by FFT length: single-pol jobs of 12 stations x 4
    subbands (64 Msps), 2^25 samples per input, N = 256 .. 32768, the library's
    default variants; kernel time per call from HIP events."""
    import torch
    from paper_1502_06894_amd import xcorr
    from synth import configs
    corr = _correlator(a)
    rows = []
    for n_chan in (128, 256, 512, 1024, 2048, 4096, 8192, 16384):
        N = 2 * n_chan
        job = configs.c4_job(device="cuda", n_stations=12, n_subbands=4, n_chan=n_chan,
                             n_frames=(1 << 25) // N)
        xcorr.job_to_device(job, "cuda:0")
        ws = corr.alloc_workspace(job)
        out = corr.alloc_output(job)
        for _ in range(a.warmup):
            corr.correlate(job, out=out, workspace=ws)
        torch.cuda.synchronize()
        corr.profile_begin(a.steps * 64 + 64)
        for _ in range(a.steps):
            corr.correlate(job, out=out, workspace=ws)
        torch.cuda.synchronize()
        prof = corr.profile_end()
        ss = job.station_samples
        f_ms, x_ms = prof["fstage"][0] / a.steps, prof["xmac"][0] / a.steps
        rows.append({"fft_len": N, "station_samples": ss, "f_ms": round(f_ms, 4),
                     "f_gss_per_s": round(ss / f_ms / 1e6, 1), "x_ms": round(x_ms, 4),
                     "x_gss_per_s": round(ss / x_ms / 1e6, 1)})
        log(f"N = {N:5d}: F {f_ms:.3f} ms ({ss / f_ms / 1e6:.1f} G ss/s), "
            f"X {x_ms:.3f} ms ({ss / x_ms / 1e6:.1f} G ss/s)")
        del ws, out, job
        torch.cuda.empty_cache()
    return {"metric": "F- and X-stage station-samples/s by FFT length", "value": None,
            "unit": "G station-samples/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "higher_is_better": True, "data": "synthetic", "dtype": "f32",
            "config": {"workload": "single-pol jobs: 12 stations x 4 subbands at 64 Msps, "
                                   "2^25 samples per input, N = 256..32768"},
            "rows": rows}


def run_fringe(a):
    """Delay-rate fringe search over a scan of C2-shaped visibilities: T = 64
    sub-integrations x 8 subbands x 210 baselines x 1024 channels, delay
    transform 2048 points, rate transform 128 points, whole-axis window."""
    import torch
    from paper_1502_06894_amd import xcorr
    T, n_sb, nbl, n_chan, D, R = 64, 8, 210, 1024, 2048, 128
    dnu, tint = 32e6 / 2048, 4.0
    g = torch.Generator(device="cuda").manual_seed(1502068946)
    V = torch.randn((T, n_sb, nbl, n_chan), dtype=torch.complex64, device="cuda", generator=g)
    d0 = torch.randint(-900, 900, (n_sb, nbl), device="cuda", generator=g).float()
    r0 = torch.randint(-50, 50, (n_sb, nbl), device="cuda", generator=g).float()
    k = torch.arange(n_chan, device="cuda").float()
    t = torch.arange(T, device="cuda").float()
    ph = 2 * np.pi * (k[None, None, None, :] * d0[None, :, :, None] / D +
                      t[:, None, None, None] * r0[None, :, :, None] / R)
    V += 0.2 * torch.polar(torch.ones_like(ph), ph)
    torch.cuda.synchronize()
    corr = xcorr.Correlator(0)
    fs = xcorr.XcFringeSetup(T, n_sb, nbl, n_chan, D, R, 0, 0, dnu, tint)
    ws = torch.empty(corr.lib.xc_fringe_workspace_bytes(ctypes_byref(fs)), dtype=torch.uint8,
                     device="cuda")
    for _ in range(a.warmup):
        peaks, _m = corr.fringe_search(V, D, R, dnu, tint, workspace=ws)
    corr.profile_begin(4 * a.steps + 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        peaks, _m = corr.fringe_search(V, D, R, dnu, tint, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    ms_k, n_k = corr.profile_end()["fringe"]
    ms_k /= max(1, a.steps)
    ok = float(np.mean((peaks["delay_bin"] == d0.cpu().numpy().astype(int)) &
                       (peaks["rate_bin"] == r0.cpu().numpy().astype(int))))
    maps = n_sb * nbl
    # per map: T delay FFTs of D points and D rate FFTs of R points (5 n log2 n
    # flops each); visibilities read once, the delay-transformed rows written and
    # read back
    flops = maps * (T * 5.0 * D * math.log2(D) + D * 5.0 * R * math.log2(R))
    bytes_ = maps * (T * n_chan * 8.0 + 2 * T * D * 8.0)
    alu = flops / (ms_k * 1e-3) / 1e12
    hbm = bytes_ / (ms_k * 1e-3) / 1e9
    log(f"fringe search: {dt * 1e3:.2f} ms per scan ({maps} maps), kernels {ms_k:.2f} ms, "
        f"{alu:.1f} TFLOP/s, {hbm:.0f} GB/s; peaks at the planted bins: {ok:.3f}")
    cpu = None
    if not a.no_cpu_baseline:
        from oracle import fringe
        # whole subband-baseline groups of 30 maps, in order, until about 10 s of CPU work
        done, dtc, t1 = 0, 0.0, time.perf_counter()
        for sb in range(n_sb):
            for b0 in range(0, nbl, 30):
                fringe.fringe_search(V[:, sb:sb + 1, b0:b0 + 30].cpu().numpy(), D, R, dnu, tint)
                done += min(30, nbl - b0)
                dtc = time.perf_counter() - t1
                if dtc > 10.0:
                    break
            if dtc > 10.0:
                break
        cpu = {"value": done / dtc, "unit": "maps/s", "cores": 1, "cpu": cpu_model(),
               "kind": "oracle",
               "sample": (f"{done} of the {maps} maps, in groups of 30 "
                          f"({dtc:.1f} s, numpy FFTs, one thread)")}
    return {
        "metric": "delay-rate maps searched/s", "value": round(maps / dt, 1), "unit": "maps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fringe search: C2-shaped scan, 64 sub-integrations x 8 subbands "
                               "x 210 baselines x 1024 channels; delay 2048, rate 128 points",
                   "maps": maps},
        "roofline": {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "fringe (delay FFT + rate FFT)",
                     "kernel_ms_per_launch": round(ms_k, 4),
                     "algorithmic_bytes_per_launch": bytes_,
                     "alu": {"achieved": round(alu, 2), "peak": FP32_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(alu / FP32_PEAK_TFLOPS, 4),
                             "flops_per_launch": flops}},
        "planted_peak_fraction": ok,
        "cpu_baseline": cpu,
    }


def run_feed(a):
    """Feed-angle correction, in place, over a C2-shaped scan of dual-pol products:
    64 sub-integrations x 8 subbands x 210 products x 1024 channels, circular feeds."""
    import torch
    from paper_1502_06894_amd import xcorr
    T, n_sb, S, n_chan = 64, 8, 10, 1024
    nbl = 2 * S * (2 * S + 1) // 2
    g = torch.Generator(device="cuda").manual_seed(1502068947)
    V = torch.randn((T, n_sb, nbl, n_chan), dtype=torch.complex64, device="cuda", generator=g)
    ang = torch.rand((T, S), dtype=torch.float64, device="cuda", generator=g) * 6.28 - 3.14
    corr = xcorr.Correlator(0)
    for _ in range(a.warmup):
        corr.feed_correct(V, ang, xcorr.XC_FEED_CIRCULAR)
    corr.profile_begin(4 * a.steps + 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        corr.feed_correct(V, ang, xcorr.XC_FEED_CIRCULAR)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    ms_k = corr.profile_end()["feed"][0] / max(1, a.steps)
    nbytes = 2.0 * V.numel() * 8                      # read and write every product
    gbs = nbytes / (ms_k * 1e-3) / 1e9
    log(f"feed correction: {dt * 1e3:.3f} ms per scan, kernel {ms_k:.3f} ms, {gbs:.0f} GB/s")
    cpu = None
    if not a.no_cpu_baseline:
        from oracle import feed
        Vh, Ah = V.cpu().numpy(), ang.cpu().numpy()
        done, dtc, t1 = 0, 0.0, time.perf_counter()
        for t in range(T):                        # one sub-integration at a time, ~10 s
            feed.correct(Vh[t:t + 1], Ah[t:t + 1], feed.CIRCULAR)
            done += 1
            dtc = time.perf_counter() - t1
            if dtc > 10.0:
                break
        cpu = {"value": done * n_sb * nbl * n_chan / dtc / 1e9, "unit": "G products/s",
               "cores": 1, "cpu": cpu_model(), "kind": "oracle",
               "sample": f"{done} of the {T} sub-integrations ({dtc:.1f} s, numpy, one thread)"}
    return {
        "metric": "feed-corrected products/s", "value": round(V.numel() / dt / 1e9, 2),
        "unit": "G products/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(dt * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "feed-angle correction: C2-shaped scan, 64 sub-integrations x 8 "
                               "subbands x 210 dual-pol products x 1024 channels, circular feeds"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "feed", "kernel_ms_per_launch": round(ms_k, 4),
                     "algorithmic_bytes_per_launch": nbytes},
        "cpu_baseline": cpu,
    }


def ctypes_byref(x):
    import ctypes
    return ctypes.byref(x)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--frames-per-block", type=int, default=0)
    ap.add_argument("--frames", type=int, default=0,
                    help="shorten the sub-integration (profiling runs only; not a bench figure)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="c2/c4: xc_tuning field override (repeatable)")
    ap.add_argument("--rate-correct", action="store_true",
                    help="c1/c2: correct the space station's delay drift inside frames")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--calibrate-read", action="store_true",
                    help="time a 4 GiB float32 sum (the device's streaming-read rate)")
    ap.add_argument("--rocpd-summary", metavar="DB", help="summarise a rocprofv3 database and exit")
    ap.add_argument("--traffic-json", nargs=4,
                    metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="write profiles/hbm_counters.json from FETCH_SIZE / WRITE_SIZE runs of "
                         "the C2 workload and of --calibrate-copy, and exit")
    ap.add_argument("--valu-json", metavar="VALU_DB",
                    help="write profiles/valu_counters.json from an SQ_INSTS_VALU + "
                         "SQ_ACTIVE_INST_VALU + GRBM_GUI_ACTIVE run of the C2 workload, and exit")
    ap.add_argument("--ss-per-launch", type=float, default=4295032832.0,
                    help="--traffic-json / --valu-json: station-samples per F / X launch of the "
                         "profiled run (C2 with --frames 13107, one default block: 10 stations x "
                         "16 inputs x 13107 frames x 2048 samples)")
    ap.add_argument("--precision", default="fp16", choices=["fp32", "fp16", "fp8"],
                    help="c4: precision reported as the value")
    ap.add_argument("--jobs", type=int, default=0, help="c3: number of jobs (64; 256 short)")
    ap.add_argument("--job-mix", default="c3", choices=["c3", "short"],
                    help="c3: the C3 mix, or many short jobs (the regime batching is for)")
    ap.add_argument("--no-autotune", action="store_true", help="c3: library default tile shapes")
    ap.add_argument("--lanes", type=int, default=0,
                    help="c3: concurrent lanes (default 8); c5: server slots (default 16)")
    ap.add_argument("--requests", type=int, default=2000, help="c5: requests in the trace")
    ap.add_argument("--check-jobs", type=int, default=50,
                    help="c5: served requests re-run alone and compared bit for bit")
    ap.add_argument("--rate", type=float, default=200.0, help="c5: mean arrival rate (1/s)")
    ap.add_argument("--max-log2-chan", type=int, default=14, help="c5: largest log2(channels)")
    ap.add_argument("--budget-gb", type=int, default=96, help="c5: server HBM budget (GiB)")
    a = ap.parse_args()
    if a.rocpd_summary:
        print(rocpd_summary(a.rocpd_summary))
        return
    if a.valu_json:
        d = valu_json(a.valu_json, a.ss_per_launch, C2_KERNELS)
        with open(os.path.join(ROOT, "profiles", "valu_counters.json"), "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d, indent=1))
        return
    if a.traffic_json:
        d = traffic_json(*a.traffic_json, a.ss_per_launch, C2_KERNELS)
        with open(os.path.join(ROOT, "profiles", "hbm_counters.json"), "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d, indent=1))
        return
    if a.gpus != 1:
        print("bench.py measures one GPU: the correlation path is built and measured on a "
              "single MI355X (multi-GPU sharding by subband x time is design-only).",
              file=sys.stderr)
        sys.exit(2)
    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.calibrate_read:
        calibrate_read()
        return

    if a.workload in ("c3", "c4", "c5", "fringe", "feed", "xcross", "fstage-n"):
        res = {"c3": run_c3, "c4": run_c4, "c5": run_c5, "fringe": run_fringe,
               "feed": run_feed, "xcross": run_xcross, "fstage-n": run_fstage_n}[a.workload](a)
        print(json.dumps(res), flush=True)
        return

    import torch
    from paper_1502_06894_amd import xcorr

    log(f"generating workload {a.workload} on the GPU")
    t = time.perf_counter()
    job, desc = make_job(a.workload, a.frames)
    if a.rate_correct:
        import dataclasses
        # the delay-drift correction on the space station (station 0)
        job = dataclasses.replace(job, stations=[dataclasses.replace(job.stations[0],
                                                                     rate_correct=True)]
                                  + list(job.stations[1:]))
        desc += "; delay-drift correction on the space station"
    xcorr.job_to_device(job, "cuda:0")
    torch.cuda.synchronize()
    log(f"workload ready in {time.perf_counter() - t:.1f} s: {job.station_samples:.3e} "
        f"station-samples per step")
    corr = _correlator(a)
    # every step runs the whole path, A0 included: the library checks each
    # recording frame's sync word (xc_ingest's kernel) inside the call
    ws = corr.alloc_workspace(job, frames_per_block=a.frames_per_block)
    out = corr.alloc_output(job)
    stream = torch.cuda.current_stream()

    def step():
        corr.correlate(job, frames_per_block=a.frames_per_block, out=out, workspace=ws,
                       stream=stream)

    for i in range(a.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({a.warmup} steps)")

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(a.steps)]
    T = a.frames_per_block or _default_fpb(job)
    blocks = -(-job.n_frames // T)
    # per block: delays, F (+ drift pass), X; per call: ingest per station, zero, finalise
    corr.profile_begin(max_launches=a.steps * (4 * blocks + job.n_stations + 4) + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = corr.profile_end()
    step_ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    dt = t1 - t0
    ss = job.station_samples
    value = ss * a.steps / dt / 1e9
    log(f"timed {a.steps} steps: {dt * 1e3 / a.steps:.2f} ms/step, {value:.1f} G ss/s")
    for k, (ms, n) in prof.items():
        if n:
            log(f"  kernel {k:9s}: {ms / a.steps:8.3f} ms/step over {n // a.steps} launches")

    # roofline of the dominant kernel: algorithmic bytes and flops per
    # station-sample (F stage: 0.25 B of 2-bit input + 4 B of FP32 spectra out;
    # 5 log2 N flops of FFT + ~10 of fringe rotation and phasor generation + ~5
    # of fractional-delay correction.  X stage: 4 B of spectra in; 2 (M + 1)
    # flops of complex multiply-accumulate)
    per_ss = {"fstage": (4.25, 5.0 * math.log2(job.N) + 15.0, F_SOURCES),
              "xmac": (4.0, 2.0 * (job.M + 1), X_SOURCES)}
    dom = max(per_ss, key=lambda k: prof[k][0])
    roof = roofline(dom, *per_ss[dom], prof[dom], ss * a.steps)
    # the other stage's record beside it (same fields)
    roof["other_stage"] = {k: roofline(k, *per_ss[k], prof[k], ss * a.steps)
                           for k in per_ss if k != dom and prof[k][1]}
    # the whole staged path against HBM: every station-sample moves 8.25 B
    roof["path_hbm"] = {"achieved": round(8.25 * value, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(8.25 * value / HBM_PEAK_GBS, 4),
                        "bytes_per_station_sample": 8.25}
    # the algorithmic figure of a fully fused path: only the 2-bit input (0.25 B
    # per station-sample) has to cross HBM
    roof["input_only_hbm"] = {"achieved": round(0.25 * value, 1), "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": round(0.25 * value / HBM_PEAK_GBS, 4),
                              "bytes_per_station_sample": 0.25}
    kernels = {k: {"ms_per_step": round(ms / a.steps, 3), "launches_per_step": n // a.steps}
               for k, (ms, n) in prof.items() if n}

    res = {
        "metric": "correlated station-samples/s",
        "value": round(value, 2),
        "unit": "G station-samples/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(dt * 1e3 / a.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "stations": job.n_stations, "subbands": job.n_subbands,
                   "pols": job.n_pols, "channels": job.n_chan, "fft_len": job.N,
                   "frames": job.n_frames, "station_samples_per_step": ss,
                   "frames_per_block": a.frames_per_block or _default_fpb(job),
                   "precision": "fp32", "parallelism": "single GPU"},
        "roofline": roof,
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                       "p99": round(float(np.percentile(step_ms, 99)), 3)},
        "kernels": kernels,
        "cpu_baseline": None,
    }
    if a.workload == "c1" and not a.rate_correct:
        # the same call as a one-job batch captured in a hipGraph: a replay
        # submits every launch of the call at once (C1 is bound by latency)
        bws = corr.batch_workspace([job], n_lanes=1)
        bouts = [corr.alloc_output(job)]
        gs = torch.cuda.Stream()
        with torch.cuda.stream(gs):
            corr.correlate_batch([job], n_lanes=1, graph=True, outs=bouts, workspace=bws,
                                 stream=gs)     # capture
            gs.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.steps):
                corr.correlate_batch([job], n_lanes=1, graph=True, outs=bouts, workspace=bws,
                                     stream=gs)
            gs.synchronize()
        tg = (time.perf_counter() - t0) / a.steps
        same = bool(torch.equal(bouts[0][0], out[0]) and torch.equal(bouts[0][1], out[1]))
        res["graph_replay"] = {"value": round(ss / tg / 1e9, 2), "ms_per_call": round(tg * 1e3, 4),
                               "identical_to_call": same}
        log(f"graph replay: {tg * 1e3:.3f} ms per call, {ss / tg / 1e9:.1f} G ss/s; "
            f"identical: {same}")
    if not a.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(job)
        log(f"oracle: {res['cpu_baseline']['value'] * 1e3:.2f} M ss/s "
            f"({res['cpu_baseline']['sample']})")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
