"""Host logic of bench.py (no GPU): the roofline record against MI355X's
published peaks, HBM traffic and VALU figures derived from rocprofv3 counter
databases (a synthetic database of the same schema), kernel-name handling, and
the consistency of the committed counter summaries the bench line reads."""
import json
import os
import sqlite3
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_roofline_names_the_roof_with_the_longer_time():
    # 2 launches of 1 ms over 2e9 station-samples: 4.25 B and 70 flop per ss
    rec = bench.roofline("no_such_kind", 4.25, 70.0, bench.F_SOURCES, (2.0, 2), 2e9)
    t = 1e-3
    t_hbm = 4.25e9 / (8000.0 * 1e9)
    t_alu = 70e9 / (157.3 * 1e12)
    assert t_hbm > t_alu
    assert rec["bound"] == "hbm" and rec["unit"] == "GB/s"
    assert rec["peak"] == 8000.0
    assert rec["frac"] == round(t_hbm / t, 4)
    assert rec["achieved"] == round(4.25e9 / t / 1e9, 1)
    assert rec["alu"]["frac"] == round(t_alu / t, 4)
    assert rec["kernel_ms_per_launch"] == 1.0 and rec["launches"] == 2
    assert rec["traffic"] is None and rec["valu_issue"] is None   # no counters for this kind
    # more flops than bytes can carry: the vector-ALU roof binds
    rec2 = bench.roofline("no_such_kind", 1.0, 200.0, bench.F_SOURCES, (1.0, 1), 1e9)
    assert rec2["bound"] == "alu" and rec2["peak"] == 157.3
    assert rec2["frac"] == round(200e9 / 157.3e12 / 1e-3, 4)
    assert rec2["hbm"]["frac"] == round(1e9 / 8e12 / 1e-3, 4)


def test_short_kernel_names():
    assert bench.short_kernel_name("void xc::k_fstage<2048, 2, 0>(xc::DevJob const*, int)") == \
        "xc::k_fstage<2048, 2, 0>"
    assert bench.short_kernel_name("xc::k_xmac_ringm<20, false>(int, (anonymous namespace)::X)") == \
        "xc::k_xmac_ringm<20, false>"


def _counter_db(path, rows):
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    db.executemany("insert into counters_collection values (?, ?, ?)", rows)
    db.commit()
    db.close()
    return str(path)


def test_traffic_and_valu_from_counter_databases(tmp_path):
    F = "void xc::k_fstage<2048, 2, 0>(xc::DevJob const*)"
    F_OTHER = "void xc::k_fstage<2048, 8, 0>(xc::DevJob const*)"   # fewer dispatches: not chosen
    X = "void xc::k_xmac_ringm<20, false>(xc::DevJob const*)"
    ss = 1.0e6
    # FETCH_SIZE / WRITE_SIZE in KiB per dispatch; the copy of 1 GiB reads as half (fetch) and
    # exactly (write), so the scales are 2 and 1
    fetch = _counter_db(tmp_path / "f.db", [(F, "FETCH_SIZE", 100.0), (F, "FETCH_SIZE", 300.0),
                                            (F_OTHER, "FETCH_SIZE", 7.0),
                                            (X, "FETCH_SIZE", 2000.0)])
    write = _counter_db(tmp_path / "w.db", [(F, "WRITE_SIZE", 4000.0), (F, "WRITE_SIZE", 4000.0),
                                            (F_OTHER, "WRITE_SIZE", 7.0),
                                            (X, "WRITE_SIZE", 50.0)])
    cfe = _counter_db(tmp_path / "cf.db", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0)])
    cwr = _counter_db(tmp_path / "cw.db", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0)])
    d = bench.traffic_json(fetch, write, cfe, cwr, ss, bench.C2_KERNELS)
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    f = d["fstage"]
    assert f["kernel"] == "xc::k_fstage<2048, 2, 0>"
    assert f["fetch_bytes_per_launch"] == round(200.0 * 2.0 * 1024)
    assert f["write_bytes_per_launch"] == round(4000.0 * 1024)
    assert f["bytes_per_station_sample"] == pytest.approx((200.0 * 2 + 4000.0) * 1024 / ss)
    assert d["xmac"]["kernel"] == "xc::k_xmac_ringm<20, false>"
    assert d["xmac"]["bytes_per_station_sample"] == pytest.approx((2000.0 * 2 + 50.0) * 1024 / ss)
    # VALU: instructions x 64 lanes per station-sample; busy over 256 CUs x one XCD's cycles;
    # matrix cores over 1024 SIMDs
    grbm = 8.0e6
    valu = _counter_db(tmp_path / "v.db", [
        (F, "SQ_INSTS_VALU", 1.0e6), (F, "SQ_ACTIVE_INST_VALU", 0.5 * 256 * grbm / 8),
        (F, "GRBM_GUI_ACTIVE", grbm), (F, "SQ_VALU_MFMA_BUSY_CYCLES", 0.0),
        (X, "SQ_INSTS_VALU", 2.0e5), (X, "SQ_ACTIVE_INST_VALU", 0.25 * 256 * grbm / 8),
        (X, "GRBM_GUI_ACTIVE", grbm), (X, "SQ_VALU_MFMA_BUSY_CYCLES", 0.4 * 1024 * grbm / 8)])
    v = bench.valu_json(valu, ss, bench.C2_KERNELS)
    assert v["fstage"]["instr_per_station_sample"] == pytest.approx(64.0)
    assert v["fstage"]["valu_busy"] == pytest.approx(0.5)
    assert v["xmac"]["instr_per_station_sample"] == pytest.approx(12.8)
    assert v["xmac"]["valu_busy"] == pytest.approx(0.25)
    assert v["xmac"]["mfma_busy"] == pytest.approx(0.4)


def test_missing_kernel_is_an_error(tmp_path):
    db = _counter_db(tmp_path / "f.db", [("void xc::k_zero(double*)", "FETCH_SIZE", 1.0)])
    with pytest.raises(SystemExit):
        bench._resolve_kernels(bench._dispatch_counts(db, "FETCH_SIZE"), bench.C2_KERNELS)


def test_committed_counter_summaries_are_consistent():
    with open(os.path.join(ROOT, "profiles", "hbm_counters.json")) as fh:
        d = json.load(fh)
    for kind in ("fstage", "xmac"):
        e = d[kind]
        per_ss = (e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]) / d["ss_per_launch"]
        assert e["bytes_per_station_sample"] == pytest.approx(per_ss, rel=1e-6)
    # the F stage writes 4 B and reads 0.25 B per station-sample; the X stage reads 4 B
    assert 4.25 <= d["fstage"]["bytes_per_station_sample"] < 4.5
    assert 4.0 <= d["xmac"]["bytes_per_station_sample"] < 4.5
    with open(os.path.join(ROOT, "profiles", "valu_counters.json")) as fh:
        v = json.load(fh)
    assert 20 < v["fstage"]["instr_per_station_sample"] < 100
    assert 0 < v["fstage"]["valu_busy"] <= 1.0


class _Shape:
    """The job fields the block-size rules read (a stand-in for a job)."""

    def __init__(self, n_subbands, M, n_chan, n_frames):
        self.n_subbands, self.M, self.n_chan, self.n_frames = n_subbands, M, n_chan, n_frames


def test_block_size_rules_mirror_the_library():
    """bench.py's copies of the library's block-size rules (the per-job check
    of the batch and served results runs each job at the block size the
    library gives it there): 2048 frames or more while a block's FP32 spectra
    stay within 16 GiB; in a batch, a 1 GiB bound unless it would cut the job
    into more than four blocks; in the server, half the budget over the slots
    (at least 1 GiB), never below 16 (M + 1) frames."""
    c2 = _Shape(8, 20, 1024, 62500)                      # 1.31 MB of spectra per frame
    assert bench._default_fpb(c2) == (16 << 30) // (8 * 20 * 1024 * 8) == 13107
    assert bench._default_fpb(_Shape(1, 2, 256, 31250)) == 31250    # small: one block
    assert bench._default_fpb(_Shape(16, 20, 8192, 5000)) == 2048    # never below 2048
    # batch: the 1 GiB bound gives C2 819 frames, 77 blocks: a long job keeps the default
    assert bench._batch_fpb(c2) == 13107
    # cut into at most four blocks by the bound: it takes the bounded size
    mid = _Shape(8, 20, 1024, 3000)
    assert bench._batch_fpb(mid) == (1 << 30) // (8 * 20 * 1024 * 8) == 819
    assert -(-mid.n_frames // 819) == 4
    # a tuned size is bounded the same way
    assert bench._batch_fpb(mid, tuned_fpb=2048) == 819
    # server: 96 GiB over 16 slots -> 3 GiB per request
    assert bench._server_fpb(c2, 96 << 30, 16) == (3 << 30) // (8 * 20 * 1024 * 8) == 2457
    # a small budget keeps the 1 GiB floor; the 16 (M + 1)-frame floor holds
    assert bench._server_fpb(c2, 4 << 30, 16) == 819
    big = _Shape(16, 40, 16384, 2000)                    # 84 MB per frame
    assert bench._server_fpb(big, 96 << 30, 16) == 16 * 41
