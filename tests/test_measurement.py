"""CPU tests of the measurement tooling: the counted-flop model of bench.py
against the oracle's own flop counter, the per-group byte figures, the
rocprofv3 summaries of paper_2301_07964_amd.profiling on small synthetic CSV
files, and the rule by which bench.py uses a committed traffic record."""
import csv
import hashlib
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2301_07964_amd import profiling as P  # noqa: E402


@pytest.mark.parametrize("n,r", [(40, 3), (64, 8), (101, 16), (200, 32)])
def test_counted_flops_model_equals_the_oracle_counter(n, r):
    """bench.py's per-class flop model (closed ranges of the unblocked
    algorithm) sums to the flops the oracle counts while it runs."""
    from oracle import oracle as O
    model = sum(bench.counted_flops_by_class(n, r).values())
    assert model == pytest.approx(O.stage2_flops(n, r), rel=1e-12)


def test_generate_bytes_per_group_is_the_band_read_and_written_once():
    # 32 n (q + 3r): H and T, read and written, 8 bytes, band of width q + 3r
    assert bench.generate_bytes_per_group(16384, 32, 32) == 32.0 * 16384 * (32 + 96)
    assert bench.generate_bytes_per_group(100, 4, 2) == 32.0 * 100 * 14


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    f = os.path.join(path, "run_counter_collection.csv")
    with open(f, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                           "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for d, k, c, v, t0, t1 in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v,
                        "Start_Timestamp": t0, "End_Timestamp": t1})
    return path


def test_short_name_drops_the_argument_list():
    assert P.short_name("void ht::k_update_mfma<32, 2, false>(ht::UpdArgs<double>, double const*)") == \
        "ht::k_update_mfma<32, 2, false>"
    assert P.short_name("ht::k_delay(long)") == "ht::k_delay"


def test_counters_sum_rows_of_one_dispatch_and_average_dispatches(tmp_path):
    # a counter reported in two rows for dispatch 1 (two XCD groups, say)
    d = _write_counters(str(tmp_path / "c"), [
        (1, "void ht::k_a(int)", "FETCH_SIZE", 10, 0, 1),
        (1, "void ht::k_a(int)", "FETCH_SIZE", 30, 0, 1),
        (2, "void ht::k_a(int)", "FETCH_SIZE", 20, 0, 1),
    ])
    c = P.counters(d)["ht::k_a"]
    assert c["dispatches"] == 2 and c["FETCH_SIZE"] == pytest.approx(30.0)


def test_traffic_scales_by_the_copy_calibration(tmp_path):
    copy_bytes = 1 << 20
    cf = _write_counters(str(tmp_path / "cf"), [(1, "copy(int)", "FETCH_SIZE", 2 * 1024, 0, 1)])   # reads x2
    cw = _write_counters(str(tmp_path / "cw"), [(1, "copy(int)", "WRITE_SIZE", 1024, 0, 1)])
    fe = _write_counters(str(tmp_path / "fe"), [(1, "ht::k_x(int)", "FETCH_SIZE", 100, 0, 1)])
    wr = _write_counters(str(tmp_path / "wr"), [(1, "ht::k_x(int)", "WRITE_SIZE", 50, 0, 1)])
    t = P.traffic(fe, wr, cf, cw, copy_bytes)
    assert t["read_factor"] == pytest.approx(0.5) and t["write_factor"] == pytest.approx(1.0)
    k = t["kernels"]["ht::k_x"]
    assert k["fetch_bytes_per_dispatch"] == pytest.approx(100 * 1024 * 0.5)
    assert k["hbm_bytes_per_dispatch"] == pytest.approx(100 * 1024 * 0.5 + 50 * 1024)


def test_mfma_table_flops_rate_and_busy_share(tmp_path):
    # one dispatch of 1 ms: 1e6 MOPS -> 5.12e8 flops -> 0.512 TFLOP/s; busy 1024 of 8 x 1024 cycles
    d = _write_counters(str(tmp_path / "m"), [
        (1, "ht::k_m(int)", "SQ_INSTS_VALU_MFMA_MOPS_F64", 1e6, 0, 1000000),
        (1, "ht::k_m(int)", "SQ_VALU_MFMA_BUSY_CYCLES", 1024, 0, 1000000),
        (1, "ht::k_m(int)", "GRBM_GUI_ACTIVE", 8 * 8, 0, 1000000),
    ])
    row = [ln for ln in P.mfma_table(d).splitlines() if "k_m" in ln][0].split("|")
    assert float(row[3]) == pytest.approx(0.51, abs=0.01)          # GFLOP per dispatch
    assert float(row[5]) == pytest.approx(0.51, abs=0.01)          # TFLOP/s
    assert float(row[7]) == pytest.approx(12.5)                    # 1024 / (8 x 1024) in percent


def test_bench_uses_a_traffic_record_only_for_unchanged_sources(tmp_path, monkeypatch):
    src = tmp_path / "k.hpp"
    src.write_text("kernel source\n")
    rec = {"kernels": {name: {"sources": [str(src)], "hbm_bytes_per_launch": 123,
                              "sources_sha256": hashlib.sha256(b"kernel source\n").hexdigest()}
                       for name in ("k_generate<double>", "k_update_mfma<left>")}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "pmc_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_generate<double>") == 123
    assert bench.measured_traffic("k_generate<double>", lookahead=1) == 123
    # the update kernels' counters are taken in the sequential schedule
    assert bench.measured_traffic("k_update_mfma<left>") == 123
    assert bench.measured_traffic("k_update_mfma<left>", lookahead=1) is None
    assert bench.measured_traffic("k_absent") is None
    src.write_text("kernel source, changed\n")
    assert bench.measured_traffic("k_generate<double>") is None


def test_streams_busy_idle_and_split(tmp_path):
    """Per-stream busy time (sum of durations), idle time (gaps between
    consecutive kernels of the stream) and the span split at a kernel."""
    from paper_2301_07964_amd import profiling as P
    f = tmp_path / "run_kernel_trace.csv"
    rows = [  # (queue, stream, name, start, end) in ns
        (1, 0, "void ht::k_s1_block_qr<double>(double*)", 0, 1_000_000),
        (1, 0, "void ht::k_s1_right_factor<double>(double*)", 1_500_000, 2_000_000),
        (1, 0, "void ht::k_s1_right_factor<double>(double*)", 2_000_000, 2_600_000),
        (2, 1, "void ht::k_s1_right_chain<double>(double*)", 1_200_000, 1_400_000),
        (2, 1, "void ht::k_s1_right_chain<double>(double*)", 2_400_000, 3_000_000),
        (1, 0, "void at::native::fill<double>(double*)", 5_000_000, 9_000_000),
    ]
    with open(f, "w") as fh:
        fh.write('"Kind","Queue_Id","Stream_Id","Kernel_Name","Start_Timestamp","End_Timestamp"\n')
        for q, st, name, b, e in rows:
            fh.write(f'"KERNEL_DISPATCH",{q},{st},"{name}",{b},{e}\n')
    r = P.streams(str(tmp_path), "k_s1", "right_factor")
    assert r["span_ms"] == pytest.approx(3.0)
    assert r["before_split_ms"] == pytest.approx(1.5) and r["after_split_ms"] == pytest.approx(1.5)
    main, side = r["streams"][("1", "0")], r["streams"][("2", "1")]
    assert main["kernels"] == 3 and main["busy_ms"] == pytest.approx(2.1) and main["idle_ms"] == pytest.approx(0.5)
    assert side["kernels"] == 2 and side["busy_ms"] == pytest.approx(0.8) and side["idle_ms"] == pytest.approx(1.0)
    assert main["names"] == {"ht::k_s1_block_qr<double>": 1, "ht::k_s1_right_factor<double>": 2}
    table = P.streams_table(str(tmp_path), "k_s1", "right_factor")
    assert "| 1 / 0 | 3 | 2.1 | 0.5 |" in table and "span 3.0 ms" in table
