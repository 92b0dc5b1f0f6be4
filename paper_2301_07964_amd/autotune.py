"""Autotuner of the stage-two paths.

Single-pencil path: the tunable is q, the number of sweeps per group (the
number of sweeps whose reflectors are generated concurrently and whose
updates are delayed together, Section 3.2); the window order of the
application kernels is 2r and their tile height follows n, so q fixes the
rest.  For each (n bucket, r) the tuner times ht_stage2_q on a synthetic r-HT
pencil for every admissible q in {r/4, r/2, r} (q >= 2) and keeps the
fastest.  Keyed "n,r" with n the bucket's upper edge; lookup() takes the
smallest bucket that holds n (beyond the largest, q = r).

Batched path (one persistent launch over many pencils): the tunable is how
a pencil is reduced, by one wavefront (64 threads, four pencils per
workgroup, no barriers) or by a workgroup of 256 threads.  For each (n
bucket, r) the tuner times a batched launch of BATCH_COUNT pencils of that
bucket (enough that either choice fills the device) under each choice and
keeps the faster; the entries (n_max, r,
threads) are handed to the library (ht_batched_set_tuning) when the binding
loads it.

Run on the GPU:  python -m paper_2301_07964_amd.autotune [--max-n N] [--out FILE] [--batched-only]
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "autotune_table.json")
BUCKETS = (64, 128, 256, 512, 1024, 2048, 4096)
RS = (4, 8, 16, 32)

_table = None


def load(path: str = TABLE):
    global _table
    if _table is None:
        _table = {}
        if os.path.exists(path):
            with open(path) as f:
                _table = json.load(f).get("q", {})
    return _table


def lookup(n: int, r: int) -> int:
    """Tuned q for (n, r); 0 (the library's built-in choice) when untuned."""
    t = load()
    for b in BUCKETS:
        if n <= b:
            return int(t.get(f"{b},{r}", 0))
    return 0


def candidates(n: int, r: int):
    re_ = min(r, max(n - 1, 1))
    out = sorted({q for q in (re_ // 4, re_ // 2, re_) if q >= 2} or {1})
    return out


def tune(max_n: int = 4096, reps: int = 2, verbose: bool = True):
    import torch
    import paper_2301_07964_amd as ht
    from paper_2301_07964_amd import inputs
    table = {}
    for b in BUCKETS:
        if b > max_n:
            break
        for r in RS:
            if r >= b / 4:
                continue
            H, T = inputs.rht_pencil(b, r, 0)
            H0, T0 = ht.colmajor(H), ht.colmajor(T)
            best = None
            for q in candidates(b, r):
                times = []
                for _ in range(reps + 1):
                    Hd, Td = H0.clone(), T0.clone()
                    Qd = torch.eye(b, dtype=torch.float64, device="cuda").t()
                    Zd = Qd.clone()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ht.stage2(Hd, Td, r, Qd, Zd, q=q)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                t = min(times[1:])
                if verbose:
                    print(f"[autotune] n={b} r={r} q={q}: {t * 1e3:.2f} ms", flush=True)
                if best is None or t < best[1]:
                    best = (q, t)
            table[f"{b},{r}"] = best[0]
    return table


BATCH_BUCKETS = (48, 64, 96, 128, 192, 256, 384, 512)
BATCH_RS = (4, 8, 16)
BATCH_COUNT = (2048, 512)        # pencils per timed launch: buckets up to 128, above (enough to fill the device)


def tune_batched(reps: int = 2, verbose: bool = True):
    """[(n_max, r, threads)] for the batched launch, per (n bucket, r)."""
    import numpy as np
    import torch
    import paper_2301_07964_amd as ht
    from paper_2301_07964_amd import inputs
    entries = []
    lo = 32
    for b in BATCH_BUCKETS:
        for r in BATCH_RS:
            if r >= lo / 4:
                continue
            rng = np.random.default_rng(b * 131 + r)
            ns = rng.integers(lo, b + 1, size=BATCH_COUNT[0] if b <= 128 else BATCH_COUNT[1])
            base = []
            for i, n in enumerate(ns):
                H, T = inputs.rht_pencil(int(n), r, i)
                base.append((ht.colmajor(H), ht.colmajor(T), r))
            best = None
            for threads in (64, 256):
                ht.set_batched_tuning([(b, 0, threads)])
                times = []
                for _ in range(reps + 1):
                    work = []
                    for H0, T0, rr in base:
                        n = H0.shape[0]
                        I = torch.eye(n, dtype=torch.float64, device="cuda").t()
                        work.append((H0.clone(memory_format=torch.preserve_format),
                                     T0.clone(memory_format=torch.preserve_format),
                                     I.clone(memory_format=torch.preserve_format),
                                     I.clone(memory_format=torch.preserve_format), rr))
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ht.stage2_batched(work)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                t = min(times[1:])
                if verbose:
                    print(f"[autotune] batched n in [{lo}, {b}] r={r} threads={threads}: {t * 1e3:.2f} ms", flush=True)
                if best is None or t < best[1]:
                    best = (threads, t)
            entries.append((b, r, best[0]))
        lo = b + 1
    ht.set_batched_tuning(entries)
    return entries


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-n", type=int, default=4096)
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--batched-only", action="store_true", help="keep the table's q entries, tune the batched path")
    a = ap.parse_args()
    old = {}
    if os.path.exists(TABLE):
        with open(TABLE) as f:
            old = json.load(f)
    t = old.get("q", {}) if a.batched_only else tune(a.max_n)
    bt = tune_batched()
    with open(a.out, "w") as f:
        json.dump({"q": t, "batched": bt,
                   "note": "q: fastest q per (n bucket, r) of the single-pencil path; batched: (n_max, r, threads) "
                           "of the persistent batched launch; measured by paper_2301_07964_amd.autotune"}, f,
                  indent=1, sort_keys=True)
    print(json.dumps({"q": t, "batched": bt}))


if __name__ == "__main__":
    main()
