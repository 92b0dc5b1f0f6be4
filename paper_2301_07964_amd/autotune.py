"""Autotuner for the single-pencil stage-two path.

The tunable is q, the number of sweeps per group (the number of sweeps whose
reflectors are generated concurrently and whose updates are delayed together,
Section 3.2); the window order of the application kernels is 2r and their
tile height follows n, so q fixes the rest.  For each (n bucket, r) the tuner
times ht_stage2_q on a synthetic r-HT pencil for every admissible q in
{r/4, r/2, r} (q >= 2) and keeps the fastest.  The table is JSON, keyed
"n,r" with n the bucket's upper edge; lookup() takes the smallest bucket
that holds n (beyond the largest, q = r).

Run on the GPU:  python -m paper_2301_07964_amd.autotune [--max-n N] [--out FILE]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-n", type=int, default=4096)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args()
    t = tune(a.max_n)
    with open(a.out, "w") as f:
        json.dump({"q": t, "note": "fastest q per (n bucket, r), measured by paper_2301_07964_amd.autotune"}, f,
                  indent=1, sort_keys=True)
    print(json.dumps(t))


if __name__ == "__main__":
    main()
