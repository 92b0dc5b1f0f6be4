"""Summaries of rocprofv3 output for the kernels of libht (measurement tooling,
not part of the reduction).

    python -m paper_2301_07964_amd.profiling stats DIR
        kernel statistics table (markdown) from DIR/run_kernel_stats.csv
    python -m paper_2301_07964_amd.profiling counters DIR
        mean counter value per dispatch, per kernel, from DIR/run_counter_collection.csv
    python -m paper_2301_07964_amd.profiling traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR COPY_BYTES
        HBM bytes per dispatch of each kernel: FETCH_SIZE and WRITE_SIZE (KiB per
        dispatch) scaled by what the same counters read for a plain device copy
        of COPY_BYTES bytes (the largest dispatch of the copy run)
    python -m paper_2301_07964_amd.profiling record FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR COPY_BYTES [NOTE]
        the same, as the record bench.py reads (profiles/pmc_traffic.json): the
        stage-two kernels of the real r = 32 path, each with the sha256 of the
        sources it is built from, so that bench.py uses a figure only while the
        kernel is unchanged; NOTE (optional) says how the counted run was made
    python -m paper_2301_07964_amd.profiling mfma DIR
        FP64 matrix-core use per kernel from a pass with SQ_INSTS_VALU_MFMA_MOPS_F64,
        SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE (markdown table)
    python -m paper_2301_07964_amd.profiling streams DIR [FILTER [SPLIT]]
        per queue and stream, from DIR/run_kernel_trace.csv: kernels, busy time
        (sum of durations) and idle time (gaps between consecutive kernels) of
        the kernels whose name contains FILTER; the span from the first to the
        last of them, split at the first kernel whose name contains SPLIT

The directories are rocprofv3 output directories written with
``--output-format csv -o run``.
"""
from __future__ import annotations

import csv
import json
import os
import re
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    """Kernel name without the argument list ('void ht::k_x<32, 2, false>(...)' -> 'ht::k_x<32, 2, false>')."""
    name = re.sub(r"^void\s+", "", name)
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def counters(path: str):
    """{kernel: {"dispatches": d, counter: mean per dispatch}} from a counter-collection CSV."""
    f = os.path.join(path, "run_counter_collection.csv") if os.path.isdir(path) else path
    vals = defaultdict(lambda: defaultdict(list))
    with open(f, newline="") as fh:
        for row in csv.DictReader(fh):
            vals[short_name(row["Kernel_Name"])][row["Counter_Name"]].append(
                (int(row["Dispatch_Id"]), float(row["Counter_Value"])))
    out = {}
    for k, cs in vals.items():
        rec = {}
        for c, lst in cs.items():
            per = defaultdict(float)
            for d, v in lst:            # a counter may come in several rows per dispatch
                per[d] += v
            rec[c] = sum(per.values()) / len(per)
            rec["dispatches"] = len(per)
        out[k] = rec
    return out


def stats_table(path: str, min_pct: float = 0.01) -> str:
    f = os.path.join(path, "run_kernel_stats.csv") if os.path.isdir(path) else path
    lines = ["| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    with open(f, newline="") as fh:
        for row in csv.DictReader(fh):
            pct = float(row["Percentage"])
            if pct < min_pct:
                continue
            lines.append(f"| `{short_name(row['Name'])}` | {row['Calls']} | {float(row['TotalDurationNs']) / 1e3:.0f} | "
                         f"{float(row['AverageNs']) / 1e3:.1f} | {pct:.2f} |")
    return "\n".join(lines)


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes):
    """HBM bytes per dispatch per kernel, scaled by the copy calibration."""
    cf, cw = counters(copy_fetch_dir), counters(copy_write_dir)

    def biggest(cs, cname):            # the copy: the dispatch family with the largest counter
        return max((rec[cname] for rec in cs.values() if cname in rec), default=0.0)

    read_factor = copy_bytes / (biggest(cf, "FETCH_SIZE") * 1024.0)
    write_factor = copy_bytes / (biggest(cw, "WRITE_SIZE") * 1024.0)
    fe, wr = counters(fetch_dir), counters(write_dir)
    out = {"read_factor": read_factor, "write_factor": write_factor, "kernels": {}}
    for k in sorted(set(fe) | set(wr)):
        fb = fe.get(k, {}).get("FETCH_SIZE", 0.0) * 1024.0 * read_factor
        wb = wr.get(k, {}).get("WRITE_SIZE", 0.0) * 1024.0 * write_factor
        out["kernels"][k] = {"dispatches": fe.get(k, {}).get("dispatches", 0),
                             "fetch_bytes_per_dispatch": fb, "write_bytes_per_dispatch": wb,
                             "hbm_bytes_per_dispatch": fb + wb}
    return out


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# bench.py's name for a kernel -> (rocprofv3 kernel name, sources it is built from)
RECORD_KERNELS = {
    "k_generate<double>": ("ht::k_generate<double, 32>",
                           ["paper_2301_07964_amd/csrc/ht_generate.hpp", "paper_2301_07964_amd/csrc/ht_common.hpp",
                            "paper_2301_07964_amd/csrc/ht_stage2.hip"]),
    "k_update_mfma<right>": ("ht::k_update_mfma<32, 2, false>",
                             ["paper_2301_07964_amd/csrc/ht_update_mfma.hpp", "paper_2301_07964_amd/csrc/ht_common.hpp",
                              "paper_2301_07964_amd/csrc/ht_stage2.hip"]),
    "k_update_mfma<left>": ("ht::k_update_mfma_coop<32, true, 1>",
                            ["paper_2301_07964_amd/csrc/ht_update_mfma.hpp", "paper_2301_07964_amd/csrc/ht_common.hpp",
                             "paper_2301_07964_amd/csrc/ht_stage2.hip"]),
}


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for src in paths:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def record(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, note=None):
    t = traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes)
    out = {"read_factor": t["read_factor"], "write_factor": t["write_factor"], "kernels": {}}
    if note:
        out["note"] = note
    for key, (kname, srcs) in RECORD_KERNELS.items():
        k = t["kernels"].get(kname)
        if not k:
            continue
        out["kernels"][key] = {"kernel_name": kname, "launches": k["dispatches"],
                               "fetch_bytes_per_launch": round(k["fetch_bytes_per_dispatch"]),
                               "write_bytes_per_launch": round(k["write_bytes_per_dispatch"]),
                               "hbm_bytes_per_launch": round(k["hbm_bytes_per_dispatch"]),
                               "sources": srcs, "sources_sha256": sources_sha256(srcs)}
    return out


def mfma_table(path: str, peak_tflops: float = 78.6, xcds: int = 8, simds: int = 1024) -> str:
    """Per kernel: FP64 MFMA flops per dispatch (MOPS x 512), the kernel's active
    time from GRBM_GUI_ACTIVE (summed over the XCDs: divided by their number,
    at the clock the run implies), executed TFLOP/s and the MFMA-busy share of
    the SIMD cycles."""
    f = os.path.join(path, "run_counter_collection.csv") if os.path.isdir(path) else path
    rows = defaultdict(lambda: defaultdict(float))
    spans = {}
    names = {}
    with open(f, newline="") as fh:
        for row in csv.DictReader(fh):
            d = int(row["Dispatch_Id"])
            rows[d][row["Counter_Name"]] += float(row["Counter_Value"])
            spans[d] = (int(row["Start_Timestamp"]), int(row["End_Timestamp"]))
            names[d] = short_name(row["Kernel_Name"])
    agg = defaultdict(lambda: defaultdict(float))
    for d, cs in rows.items():
        a = agg[names[d]]
        a["n"] += 1
        a["flops"] += cs.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512.0
        a["busy"] += cs.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        a["active"] += cs.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        a["ns"] += spans[d][1] - spans[d][0]
    lines = ["| kernel | dispatches | FP64 MFMA GFLOP per dispatch | mean dispatch ms | executed TFLOP/s | % of "
             f"{peak_tflops} | MFMA busy % of SIMD cycles |", "|---|---|---|---|---|---|---|"]
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["flops"]):
        if a["flops"] <= 0:
            continue
        tf = a["flops"] / (a["ns"] * 1e-9) / 1e12
        lines.append(f"| `{k}` | {int(a['n'])} | {a['flops'] / a['n'] / 1e9:.2f} | {a['ns'] / a['n'] / 1e6:.3f} | "
                     f"{tf:.2f} | {100 * tf / peak_tflops:.1f} | {100 * a['busy'] / (a['active'] * simds):.1f} |")
    return "\n".join(lines)


def streams(path: str, match: str = "", split: str | None = None):
    """Per-stream occupancy of the kernels whose name contains `match`, from a
    kernel-trace CSV: {"span_ms", "before_split_ms", "after_split_ms",
    "streams": {(queue, stream): {"kernels", "busy_ms", "idle_ms", "names"}}}."""
    f = os.path.join(path, "run_kernel_trace.csv") if os.path.isdir(path) else path
    rows = []
    with open(f, newline="") as fh:
        for row in csv.DictReader(fh):
            if match in row["Kernel_Name"]:
                rows.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"]), row["Queue_Id"],
                             row["Stream_Id"], short_name(row["Kernel_Name"])))
    if not rows:
        return {"span_ms": 0.0, "streams": {}}
    rows.sort()
    t0, t1 = rows[0][0], max(r[1] for r in rows)
    out = {"span_ms": (t1 - t0) / 1e6, "streams": {}}
    if split:
        ts = next((r[0] for r in rows if split in r[4]), None)
        if ts is not None:
            out["before_split_ms"] = (ts - t0) / 1e6
            out["after_split_ms"] = (t1 - ts) / 1e6
    per = defaultdict(list)
    for r in rows:
        per[(r[2], r[3])].append(r)
    for key, lst in sorted(per.items()):
        busy = sum(e - b for b, e, *_ in lst)
        idle = sum(max(0, b2 - e1) for (_, e1, *_), (b2, *_) in zip(lst, lst[1:]))
        names = defaultdict(int)
        for r in lst:
            names[r[4]] += 1
        out["streams"][key] = {"kernels": len(lst), "busy_ms": busy / 1e6, "idle_ms": idle / 1e6,
                               "names": dict(names)}
    return out


def streams_table(path: str, match: str = "", split: str | None = None) -> str:
    r = streams(path, match, split)
    head = f"span {r['span_ms']:.1f} ms"
    if "before_split_ms" in r:
        head += f" ({r['before_split_ms']:.1f} ms before the first {split}, {r['after_split_ms']:.1f} ms from it)"
    lines = [head, "", "| queue / stream | kernels | busy ms | idle ms | kernels by name |", "|---|---|---|---|---|"]
    for (q, st), a in r["streams"].items():
        names = ", ".join(f"`{k}` {v}" for k, v in sorted(a["names"].items()))
        lines.append(f"| {q} / {st} | {a['kernels']} | {a['busy_ms']:.1f} | {a['idle_ms']:.1f} | {names} |")
    return "\n".join(lines)


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(stats_table(argv[1]))
    elif len(argv) >= 2 and argv[0] == "counters":
        print(json.dumps(counters(argv[1]), indent=1))
    elif len(argv) >= 6 and argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2], argv[3], argv[4], float(argv[5])), indent=1))
    elif len(argv) >= 6 and argv[0] == "record":
        print(json.dumps(record(argv[1], argv[2], argv[3], argv[4], float(argv[5]),
                                argv[6] if len(argv) > 6 else None), indent=1))
    elif len(argv) >= 2 and argv[0] == "mfma":
        print(mfma_table(argv[1]))
    elif len(argv) >= 2 and argv[0] == "streams":
        print(streams_table(argv[1], argv[2] if len(argv) > 2 else "", argv[3] if len(argv) > 3 else None))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
