#!/usr/bin/env python
"""Stage-two Hessenberg-triangular reduction throughput on one MI355X.

Default workload: one real FP64 r-Hessenberg-triangular pencil, n = 16384,
r = 32, seed 0, Q and Z accumulated (the configuration the headline metric is
quoted on).  A step is one full stage-two reduction ``ht_stage2`` of one
pencil.  The inputs of every step are restored in HBM from pristine device
copies before the step (outside the timed region); the timed region is the sum
over exactly ``--steps`` reductions, each bracketed by device
synchronisation.

Prints ONE JSON line: the metric (counted-flop GFLOP/s, see below), the
roofline record of the dominant kernel (measured live with HIP events on the
stream the kernels run on) and the CPU oracle timed on a bounded sample of the
same workload on the host cores.

Counted flops: 4 x reflector length x vectors updated for every reflector
application of the unblocked algorithm (the paper's Section 3.1 states 10 n^3;
the exact count of its algorithm is 8.0 n^3 + O(r n^2), 3.525e13 here).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
HBM_PEAK_GBS = 8000.0


def generate_band_bytes(n, r, q, esz=8):
    """Algorithmic HBM bytes of the generate phase, per group (list over the
    groups): the band of H and T that the generate phase of Section 3.2 updates,
    each entry read and written once per group.  Ranges of the right reflector
    of step (j, k) (the generate algorithm of the appendix, with the top rows
    derived for the grouped order, d = j2 - j): rows
    max(j1+1, j1+1+(k+1-d) r) .. min(j+(k+2)r, n) of H and
    max(j1+1, j1+1+(k-d) r) .. min(j+(k+1)r, n) of T in the block's columns.
    Per column the band is the union of the row ranges of the steps whose
    block holds it.  1-based indices as in the paper."""
    import numpy as np
    out = []
    c = np.arange(1, n + 1, dtype=np.int64)          # 1-based columns
    for j1 in range(1, n - 1, q):
        j2 = min(j1 + q - 1, n - 2)
        topH = np.full(n, n + 1, dtype=np.int64)
        topT = np.full(n, n + 1, dtype=np.int64)
        botH = np.zeros(n, dtype=np.int64)
        botT = np.zeros(n, dtype=np.int64)
        for j in range(j1, j2 + 1):
            if n - j - 2 < 0:
                continue
            nb = 1 + (n - j - 2) // r
            d = j2 - j
            k = (c - j - 1) // r                         # block of sweep j holding column c
            on = (c >= j + 1) & (k < nb)
            i2 = np.minimum(j + (k + 1) * r, n)
            i3 = np.minimum(j + (k + 2) * r, n)
            tH = np.maximum(j1 + 1, j1 + 1 + (k + 1 - d) * r)
            tT = np.maximum(j1 + 1, j1 + 1 + (k - d) * r)
            topH = np.where(on, np.minimum(topH, tH), topH)
            topT = np.where(on, np.minimum(topT, tT), topT)
            botH = np.where(on, np.maximum(botH, i3), botH)
            botT = np.where(on, np.maximum(botT, i2), botT)
        rows = np.where(botH > 0, botH - topH + 1, 0) + np.where(botT > 0, botT - topT + 1, 0)
        out.append(float(rows.sum()) * 2 * esz)
    return out


def counted_flops_by_class(n, r):
    """Algorithmic flops of the unblocked algorithm, split by the kernel class
    of the blocked implementation that performs them: right updates of H and T
    (rows 1..i3 of H, 1..i2 of T), updates of Q and Z (all n rows each) and
    left updates of H and T (columns jb..n of H, i1..n of T, the ranges the
    algorithm states)."""
    import numpy as np
    right = qz = left = 0.0
    for j in range(1, n - 1):
        nb = 1 + (n - j - 2) // r
        k = np.arange(nb, dtype=np.int64)
        jb = j + np.maximum(0, (k - 1) * r + 1)
        i1 = j + k * r + 1
        i2 = np.minimum(j + (k + 1) * r, n)
        i3 = np.minimum(j + (k + 2) * r, n)
        m = (i2 - i1 + 1).astype(np.float64)
        right += float(np.sum(4.0 * m * (i3 + i2)))
        qz += float(np.sum(4.0 * m * 2.0 * n))
        left += float(np.sum(4.0 * m * ((n - jb + 1) + (n - i1 + 1))))
    return {"update_right": right, "update_qz": qz, "update_left": left}


def update_bytes_by_class(n, r, q):
    """Algorithmic HBM bytes of the application kernels: every matrix entry a
    group's delayed updates change is read and written once (16 B per real
    entry), with the row/column ranges of the streaming windows (window k of a
    group starting at sweep j1 spans columns j1+k*r .. j1+k*r+W-1, 0-based,
    W = q+r-1; H rows up to the window bottom + (q+2)r, T + (q+1)r, Q and Z all
    rows; left updates of H and T from column lo_k - (q+1)r on)."""
    right = qz = left = 0.0
    for j1 in range(1, n - 1, q):
        j2 = min(j1 + q - 1, n - 2)
        qg = j2 - j1 + 1
        kmax = 1 + (n - j1 - 2) // r
        W = qg + r - 1
        for k in range(kmax):
            lo = j1 + k * r
            hi = min(lo + W - 1, n - 1)
            new = (min(n, lo + W) - lo) if k == kmax - 1 else (min(n, lo + r) - lo)
            right += new * (min(n, hi + 1 + (q + 2) * r) + min(n, hi + 1 + (q + 1) * r))
            qz += new * 2 * n
            left += new * 2 * (n - max(0, lo - (q + 1) * r))
    return {"update_right": 16.0 * right, "update_qz": 16.0 * qz, "update_left": 16.0 * left}


def update_mfma_flops_by_class(n, r, q):
    """Flops the matrix-core application kernels execute: every line (row for
    right updates, column for left updates) a window reaches is multiplied by
    the window's dense orthogonal factor of order KW = max(16, 2r), 2 KW^2
    flops, with the line ranges of update_bytes_by_class."""
    KW = max(16, 2 * r)
    right = qz = left = 0.0
    for j1 in range(1, n - 1, q):
        kmax = 1 + (n - j1 - 2) // r
        W = min(q, n - 1 - j1) + r - 1
        for k in range(kmax):
            lo = j1 + k * r
            hi = min(lo + W - 1, n - 1)
            right += min(n, hi + 1 + (q + 2) * r) + min(n, hi + 1 + (q + 1) * r)
            qz += 2 * n
            left += 2 * (n - max(0, lo - (q + 1) * r))
    f = 2.0 * KW * KW
    return {"update_right": f * right, "update_qz": f * qz, "update_left": f * left}


def cpu_baseline(H, T, r, target_s=20.0):
    """The oracle on the host cores (its threaded form, bitwise equal to one
    thread): the first s sweeps of the same pencil, s sized for about
    target_s seconds of work from two timed prefixes (2 and 6 sweeps), which
    separate the per-sweep time from the fixed cost of a call (copying H, T
    and the identity Q, Z in).  The per-sweep estimate is held at no less
    than 1/40 of the 6-sweep call, so that timing noise cannot size the
    sample far beyond target_s."""
    from oracle import oracle as O
    # the host's share of cores: the affinity mask, capped by OMP_NUM_THREADS
    # where the machine sets it
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    cores = max(1, min(O.host_cores(), cap if cap > 0 else 64, 64))
    old = O.set_threads(cores)

    def timed(jmax):
        print(f"[bench] cpu oracle: first {jmax} sweeps on {cores} threads", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        res = O.stage2(H, T, r, jmax=jmax)
        return time.perf_counter() - t0, res

    try:
        t2, _ = timed(2)
        t6, _ = timed(6)
        per = max((t6 - t2) / 4, t6 / 40)
        fixed = max(t2 - 2 * per, 0.0)
        s = max(1, min(H.shape[0] - 2, int((target_s - fixed) / per)))
        ts, res = timed(s)
        fs = res[4]
    finally:
        O.set_threads(old)
    return {"value": round(fs / ts / 1e9, 4), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"first {s} of {H.shape[0] - 2} sweeps of the same pencil (counted flops {fs:.3e}, "
                      f"{ts:.1f} s including the copy-in of H, T and the identity Q, Z; {cores} threads)"}


def generate_bytes_per_group(n, r, q):
    """Algorithmic HBM bytes of one generate launch (one group of q sweeps):
    the diagonal band of H and T of width about q+3r that the generation
    works on, read and written once, 2 matrices x 2 directions x 8 B:
    32 n (q + 3r)."""
    return 32.0 * n * (q + 3 * r)


def bench_batched(args):
    """2048 independent r-HT pencils (n uniform on [32, 512], r in {4, 8, 16}
    with r < n/4, Q and Z accumulated): one persistent ht_stage2_batched
    launch vs a loop of single ht_stage2 calls (q from the autotune table) on
    one stream.  Reports pencils/s of both and the p50/p99 completion time of
    the pencils inside the persistent launch (device clock)."""
    import numpy as np
    import torch
    import paper_2301_07964_amd as ht
    from paper_2301_07964_amd import autotune, inputs

    cnt = args.count
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = inputs.batch_configs(cnt, args.seed)
    print(f"[bench] generating {cnt} pencils", file=sys.stderr, flush=True)
    base = []
    for b, (n, r) in enumerate(cfg):
        H, T = inputs.rht_pencil(n, r, args.seed * 1000003 + b)
        base.append((ht.colmajor(H, dev), ht.colmajor(T, dev), r))
    flops = 0.0
    for (n, r) in cfg:
        flops += sum(counted_flops_by_class(n, r).values())

    def fresh():
        out = []
        for H0, T0, r in base:
            n = H0.shape[0]
            I = torch.eye(n, dtype=torch.float64, device=dev).t()
            out.append((H0.clone(memory_format=torch.preserve_format), T0.clone(memory_format=torch.preserve_format),
                        I.clone(memory_format=torch.preserve_format), I.clone(memory_format=torch.preserve_format), r))
        return out

    stream = torch.cuda.current_stream()
    # warm-up, then the timed persistent launch (kernel timing on for the stamps)
    ht.stage2_batched(fresh()[:64], stream=stream)
    torch.cuda.synchronize()
    work = fresh()
    torch.cuda.synchronize()
    ht.profile_enable(True)
    t0 = time.perf_counter()
    ht.stage2_batched(work, stream=stream)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    ht.profile_enable(False)
    done = np.array(ht.batched_completion_ms(cnt))
    ht.profile_read()
    print(f"[bench] persistent launch: {t_batched:.3f} s", file=sys.stderr, flush=True)

    # invariants on every pencil of the batched run
    worst = 0.0
    eps = float(np.finfo(np.float64).eps)
    ok = True
    for (Hd, Td, Qd, Zd, r), (H0, T0, _) in zip(work, base):
        n = Hd.shape[0]
        I = torch.eye(n, dtype=torch.float64, device=dev)
        e = max(torch.linalg.norm(Qd.t() @ Qd - I).item(), torch.linalg.norm(Zd.t() @ Zd - I).item(),
                (torch.linalg.norm(Qd @ Hd @ Zd.t() - H0) / torch.linalg.norm(H0)).item(),
                (torch.linalg.norm(Qd @ Td @ Zd.t() - T0) / torch.linalg.norm(T0)).item())
        zeros = bool((torch.tril(Hd, -2) == 0).all().item() and (torch.tril(Td, -1) == 0).all().item())
        ok = ok and zeros and e <= 100 * n * eps
        worst = max(worst, e / (n * eps))
    del work

    # loop of single launches on one stream (autotuned q)
    work = fresh()
    torch.cuda.synchronize()
    print(f"[bench] loop of {cnt} single launches", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for i, (Hd, Td, Qd, Zd, r) in enumerate(work):
        ht.stage2(Hd, Td, r, Qd, Zd, q=autotune.lookup(Hd.shape[0], r), stream=stream)
        if (i + 1) % 512 == 0:
            torch.cuda.synchronize()
            print(f"[bench]   {i + 1} done, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    del work

    out = {
        "metric": "batched pencils/s (2048 r-HT pencils, one persistent launch) + p99 latency",
        "value": round(cnt / t_batched, 1),
        "unit": "pencils/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(t_batched * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cnt} independent r-HT pencils, n uniform on [32, 512], r in {{4, 8, 16}} with r < n/4, "
                               f"Q and Z accumulated, seed {args.seed}", "count": cnt},
        "counted_gflops_per_s": round(flops / t_batched / 1e9, 2),
        "loop_of_single_launches": {"pencils_per_s": round(cnt / t_loop, 2), "seconds": round(t_loop, 3),
                                    "q": "autotune table"},
        "speedup_vs_loop": round(t_loop / t_batched, 2),
        "completion_ms": {"p50": round(float(np.percentile(done, 50)), 3),
                          "p99": round(float(np.percentile(done, 99)), 3),
                          "max": round(float(done.max()), 3), "clock": "device wall clock, from the first pencil start"},
        "check": {"ok": ok, "worst_error_over_n_eps": round(worst, 3), "bound_over_n_eps": 100},
    }
    print(json.dumps(out))


def bench_serving(args):
    """Complex128 request stream: n log-uniform on [64, 8192], r in {8, 16, 32}
    with r < n/4, 20% dense (stage one first), Poisson arrivals.  Two arrival
    rates: 0.8 x the FIFO capacity and 0.8 x the continuous-batching capacity,
    both measured on a calibration sample (all arriving at once) in the same
    run; both policies replay the same trace at each rate.  Reports p50/p99
    latency (completion - arrival, host clock, queueing included) and
    pencils/s.  (Served results are checked against the oracle and against
    the same request reduced alone in the GPU tests.)"""
    import numpy as np
    # one hardware queue per execution stream (6 slots x 2 streams + the batch
    # stream); HIP reads this when it initialises, below
    os.environ["GPU_MAX_HW_QUEUES"] = "16"
    import torch
    import paper_2301_07964_amd.serving as S

    torch.cuda.set_device(0)
    count = args.count if args.count != 2048 else 40
    # calibration: a sample that arrives at once, served by each policy
    caps = {}
    for policy in ("fifo", "continuous"):
        cal = S.make_trace(12, rate=0.0, seed=args.seed + 1)
        print(f"[bench] calibration ({policy}): {len(cal)} requests, n={[q.n for q in cal]}", file=sys.stderr,
              flush=True)
        t0 = time.perf_counter()
        S.Engine(policy).run(cal, time_limit=1200, progress=lambda k, tot, now, p=policy: print(
            f"[bench] calibration ({p}): {k}/{tot} done at {now:.1f} s", file=sys.stderr, flush=True))
        caps[policy] = len(cal) / (time.perf_counter() - t0)
    print(f"[bench] capacities: {caps}", file=sys.stderr, flush=True)
    points = []
    for label, lam in (("0.8 x FIFO capacity", 0.8 * caps["fifo"]),
                       ("0.8 x continuous-batching capacity", 0.8 * caps["continuous"])):
        res = {}
        for policy in ("fifo", "continuous"):
            trace = S.make_trace(count, rate=lam, seed=args.seed)
            eng = S.Engine(policy)
            t0 = time.perf_counter()

            def progress(k, tot, now, policy=policy):
                print(f"[bench] {label}, {policy}: {k}/{tot} requests done at {now:.1f} s", file=sys.stderr,
                      flush=True)
            eng.run(trace, time_limit=1500, progress=progress)
            wall = time.perf_counter() - t0
            res[policy] = dict(S.summary(trace), wall_s=round(wall, 3), max_inflight=eng.max_inflight,
                               peak_accounted_gb=round(eng.peak_bytes / 2 ** 30, 2))
            print(f"[bench] {label}, {policy}: {res[policy]}", file=sys.stderr, flush=True)
        points.append({"arrival": label, "rate_per_s": round(lam, 4), "fifo": res["fifo"],
                       "continuous": res["continuous"],
                       "p99_ratio_fifo_over_continuous": round(res["fifo"]["p99_ms"] / res["continuous"]["p99_ms"], 3),
                       "p50_ratio_fifo_over_continuous": round(res["fifo"]["p50_ms"] / res["continuous"]["p50_ms"], 3)})
    c = points[0]["continuous"]
    out = {
        "metric": "serving: p99 latency and pencils/s of continuous batching vs one-pencil-per-launch FIFO",
        "value": c["p99_ms"],
        "unit": "ms (p99 latency, continuous batching, arrivals at 0.8 x FIFO capacity)",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(c["wall_s"] * 1e3, 1),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"{count} complex128 reduction requests, n log-uniform on [64, 8192], r in {{8, 16, 32}}, "
                               f"20% dense, Poisson arrivals, seed {args.seed}",
                   "capacity_fifo": round(caps["fifo"], 4), "capacity_continuous": round(caps["continuous"], 4),
                   "hbm_budget": "0.8 x free HBM"},
        "points": points,
    }
    print(json.dumps(out))


def bench_stage1(args):
    """Stage one alone (ht_rhess / ht_rhess_z): a dense pencil with i.i.d.
    N(0,1) (complex: CN(0,1)) entries reduced to r-HT form with Q and Z
    accumulated.  Flops: the QR of B (about (4/3 + 2 + 4/3) n^3 with the
    application to A and the forming of Q) plus (28p+14)/(3(p-1)) n^3 for the
    panels, times 4 for complex."""
    import numpy as np
    import torch
    import paper_2301_07964_amd as ht
    from paper_2301_07964_amd import inputs
    n, r, cplx = args.n, args.r, args.complex
    ht.set_knob(ht.KNOB_LOOKAHEAD, args.lookahead)
    A, B = inputs.dense_pencil(n, seed=args.seed, complex_=cplx)
    A0, B0 = ht.colmajor(A), ht.colmajor(B)
    del A, B
    eye = torch.eye(n, dtype=A0.dtype, device=A0.device)
    p = ht.rhess_default_p(n, r)
    times = []
    for it in range(args.warmup + args.steps):
        Ad, Bd = A0.clone(), B0.clone()
        Qd = eye.t().contiguous().t().clone()
        Zd = Qd.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ht.rhess(Ad, Bd, r, Qd, Zd)
        torch.cuda.synchronize()
        if it >= args.warmup:
            times.append(time.perf_counter() - t0)
        print(f"[bench] stage one step {it + 1}/{args.warmup + args.steps}: {time.perf_counter() - t0:.3f} s",
              file=sys.stderr, flush=True)
    t = sum(times) / len(times)
    flops = ((4.0 / 3.0 + 2.0 + 4.0 / 3.0) + (28 * p + 14) / (3.0 * (p - 1))) * float(n) ** 3 * (4 if cplx else 1)
    nb = min(r, n - 1)
    check = None
    if not args.no_check:
        I = torch.eye(n, dtype=A0.dtype, device=A0.device)
        ii = torch.arange(n, device=A0.device)
        check = {"pattern_A": bool((Ad.abs() * (ii[:, None] > ii[None, :] + nb)).max().item() == 0),
                 "pattern_B": bool((Bd.abs() * (ii[:, None] > ii[None, :])).max().item() == 0),
                 "orth_Q": torch.linalg.norm(Qd.conj().t() @ Qd - I).item(),
                 "backward_A": (torch.linalg.norm(Qd @ Ad @ Zd.conj().t() - A0) / torch.linalg.norm(A0)).item(),
                 "backward_B": (torch.linalg.norm(Qd @ Bd @ Zd.conj().t() - B0) / torch.linalg.norm(B0)).item()}
    print(json.dumps({"metric": "stage-one (dense -> r-HT) GFLOP/s", "value": round(flops / t / 1e9, 2),
                      "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(t * 1e3, 2), "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "c128" if cplx else "f64", "data": "synthetic",
                      "config": {"workload": f"stage one of a dense {'complex128' if cplx else 'FP64'} pencil, n={n}, "
                                             f"r={r} (p={p}), Q and Z accumulated, seed {args.seed}",
                                 "n": n, "r": r, "p": p, "lookahead": args.lookahead},
                      "flops_per_step": flops, "check": check}))


def bench_copy(args):
    """A plain device-to-device copy of a known size (the calibration kernel
    for the FETCH_SIZE / WRITE_SIZE counters: bytes counted per byte moved)."""
    import torch
    nbytes = args.copy_bytes
    n = nbytes // 8
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / max(args.steps, 1)
    print(json.dumps({"metric": "device copy bandwidth (counter calibration)", "value": round(2 * n * 8 / t / 1e9, 1),
                      "unit": "GB/s", "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                      "steps": args.steps, "warmup": args.warmup, "n_gpus": 1}))


def measured_traffic(kernel: str, lookahead: int = 0):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/pmc_traffic.json), if it was taken on the current source of the
    kernel; None otherwise.  The counters are taken with the groups in
    sequence (counter collection runs one kernel at a time); with lookahead
    the left pass also does the band copy and the exact zeros, and the H/T
    right pass runs in another kernel (the four-wavefront tiles), so the
    update kernels' figures do not apply and None is returned for them."""
    if lookahead and kernel != "k_generate<double>":
        return None
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    h = hashlib.sha256()
    for src in k.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != k.get("sources_sha256"):
        return None
    return k.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--r", type=int, default=32)
    ap.add_argument("--q", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--workload", choices=("single", "batched", "serving", "stage1", "copy"), default="single",
                    help="single: one n x n pencil (headline); batched: 2048 small pencils in one launch; "
                         "serving: the complex128 request loop; stage1: dense -> r-HT; copy: counter calibration")
    ap.add_argument("--complex", action="store_true", help="stage1: complex128 pencil")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--count", type=int, default=2048, help="batched: number of pencils")
    ap.add_argument("--lookahead", type=int, choices=(0, 1, 2), default=1,
                    help="single: 1 (the default) overlaps each group's generation with the previous group's left "
                         "pass from n = 1024 on, 2 at every n, 0 runs the groups one after the other (for "
                         "profilers that run one kernel at a time, where the overlapped schedule would wait on a "
                         "kernel that cannot start); stage1: the same values switch the three-stream schedule")
    ap.add_argument("--wait-polls", type=int, default=0,
                    help="single: polls before a device-side wait gives up (0: the library default)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported "
              "(the reduction of one pencil is not sharded across devices).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "stage1":
        return bench_stage1(args)

    import numpy as np
    import torch
    import paper_2301_07964_amd as ht
    from paper_2301_07964_amd import inputs

    n, r = args.n, args.r
    K, W = args.steps, args.warmup
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] generating r-HT pencil n={n} r={r} seed={args.seed}", file=sys.stderr, flush=True)
    H, T = inputs.rht_pencil(n, r, args.seed)
    Hd0, Td0 = ht.colmajor(H, dev), ht.colmajor(T, dev)
    q = args.q if args.q else ht.default_q(n, r)
    # one working set, restored from the pristine copies before every step
    # (outside the timed region)
    Hd, Td = torch.empty_like(Hd0), torch.empty_like(Td0)
    Qd = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device=dev)
    Zd = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device=dev)

    def restore():
        Hd.copy_(Hd0)
        Td.copy_(Td0)
        for X in (Qd, Zd):
            X.zero_()
            X.diagonal().fill_(1.0)
        torch.cuda.synchronize()

    ht.set_knob(ht.KNOB_LOOKAHEAD, args.lookahead)
    if args.wait_polls > 0:
        ht.set_knob(ht.KNOB_WAIT_POLLS, args.wait_polls)
    stream = torch.cuda.current_stream()
    for i in range(W):
        print(f"[bench] warmup {i + 1}/{W}", file=sys.stderr, flush=True)
        restore()
        ht.stage2(Hd, Td, r, Qd, Zd, q=q, stream=stream)
        torch.cuda.synchronize()

    ht.profile_enable(True)
    elapsed = 0.0
    for i in range(K):
        restore()
        t0 = time.perf_counter()
        ht.stage2(Hd, Td, r, Qd, Zd, q=q, stream=stream)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        print(f"[bench] step {i + 1}/{K}: {time.perf_counter() - t0:.3f} s", file=sys.stderr, flush=True)
    ht.profile_enable(False)
    prof = ht.profile_read()
    status = ht.stream_status(stream)
    print(f"[bench] {K} steps in {elapsed:.3f} s; kernel ms: "
          + ", ".join(f"{k}={v[0]:.1f}/{v[1]}" for k, v in prof.items()), file=sys.stderr, flush=True)

    per_class_flops = counted_flops_by_class(n, r)
    total_flops = sum(per_class_flops.values())
    value = total_flops * K / elapsed / 1e9

    # Roofline of the dominant kernel (by total time over the timed region).
    # The application kernels stream every entry they update once per group
    # (about q/4 algorithmic flop per byte, below the FP64 ridge 78.6/8 = 9.8):
    # HBM bound.  Generation is a latency-bound pipeline; its algorithmic bytes
    # are the band it updates, read and written once per group.
    per_class_bytes = update_bytes_by_class(n, r, q)
    per_class_exec = update_mfma_flops_by_class(n, r, q)
    mfma = r in (4, 8, 16, 32)
    kernels = {("k_update_mfma<right>" if mfma else "k_update_right_reg<double>"): ("update_right", "update_qz"),
               ("k_update_mfma<left>" if mfma else "k_update_left_reg<double>"): ("update_left",),
               "k_generate<double>": ("generate",)}
    ktime = {kn: sum(prof[c][0] for c in cl) for kn, cl in kernels.items()}
    klaunch = {kn: sum(prof[c][1] for c in cl) for kn, cl in kernels.items()}
    dom = max(ktime, key=ktime.get)
    updates = {}
    for kn, cl in kernels.items():
        if kn == "k_generate<double>" or klaunch[kn] == 0:
            continue
        mean_s = ktime[kn] / klaunch[kn] * 1e-3
        b = sum(per_class_bytes[c] for c in cl) * K / klaunch[kn]
        f = sum(per_class_flops[c] for c in cl) * K / klaunch[kn]
        fx = sum(per_class_exec[c] for c in cl) * K / klaunch[kn]
        updates[kn] = {"mean_launch_ms": round(mean_s * 1e3, 4), "launches": klaunch[kn],
                       "hbm_gbs": round(b / mean_s / 1e9, 1), "hbm_frac": round(b / mean_s / 1e9 / HBM_PEAK_GBS, 4),
                       "algorithmic_tflops": round(f / mean_s / 1e12, 3),
                       "mfma_executed_tflops": round(fx / mean_s / 1e12, 3) if mfma else None,
                       "mfma_frac": round(fx / mean_s / 1e12 / FP64_PEAK_TFLOPS, 4) if mfma else None,
                       "traffic": measured_traffic(kn, args.lookahead)}
    if dom != "k_generate<double>" and klaunch[dom] > 0:
        u = updates[dom]
        per_launch_b = sum(per_class_bytes[c] for c in kernels[dom]) * K / klaunch[dom]
        achieved = per_launch_b / (u["mean_launch_ms"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": u["traffic"], "kernel": dom,
                    "algorithmic_bytes_per_launch": per_launch_b,
                    "mean_launch_ms": u["mean_launch_ms"], "launches": klaunch[dom]}
    else:
        launches = max(klaunch[dom], 1)
        per_launch_b = generate_bytes_per_group(n, r, q)
        mean_s = ktime[dom] / launches * 1e-3
        achieved = per_launch_b / mean_s / 1e9
        band = generate_band_bytes(n, r, q)
        roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": measured_traffic(dom, args.lookahead), "kernel": dom,
                    "algorithmic_bytes_per_launch": per_launch_b,
                    "algorithmic_bytes": "32 n (q + 3r) per group: the band of width q+3r of H and T, read and "
                                         "written once",
                    "eager_range_bytes_per_launch": sum(band) / max(len(band), 1),
                    "mean_launch_ms": round(mean_s * 1e3, 4), "launches": klaunch[dom]}
    roofline["by_kernel_ms"] = {kn: round(v, 2) for kn, v in ktime.items()}

    check = None
    if not args.no_check:
        eps = float(np.finfo(np.float64).eps)
        Hr = torch.tril(Hd, -2).abs().max().item() if n > 2 else 0.0
        Tr = torch.tril(Td, -1).abs().max().item() if n > 1 else 0.0
        I = torch.eye(n, dtype=torch.float64, device=dev)
        orth_q = torch.linalg.norm(Qd.t() @ Qd - I).item()
        orth_z = torch.linalg.norm(Zd.t() @ Zd - I).item()
        bH = (torch.linalg.norm(Qd @ Hd @ Zd.t() - Hd0) / torch.linalg.norm(Hd0)).item()
        bT = (torch.linalg.norm(Qd @ Td @ Zd.t() - Td0) / torch.linalg.norm(Td0)).item()
        bound = 100 * n * eps
        check = {"exact_zeros": Hr == 0.0 and Tr == 0.0, "orth_Q": orth_q, "orth_Z": orth_z,
                 "backward_H": bH, "backward_T": bT, "bound_100neps": bound,
                 "device_status": status,
                 "ok": status == 0 and Hr == 0.0 and Tr == 0.0 and max(orth_q, orth_z, bH, bT) <= bound}
        del I

    cpu = None
    if not args.no_cpu:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(H, T, r, args.cpu_seconds)

    out = {
        "metric": "stage-2 HT FP64 GFLOP/s + % FP64 peak at n=16384; batched pencils/s, p99 latency",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(elapsed / K * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"stage-2 reduction of one r-HT pencil, n={n}, r={r}, Q and Z accumulated, seed {args.seed}",
                   "n": n, "r": r, "q": q, "seed": args.seed, "lookahead": args.lookahead},
        "pct_fp64_peak": round(value / (FP64_PEAK_TFLOPS * 1e3) * 100, 3),
        "counted_flops_per_step": total_flops,
        "kernel_ms": {k: round(v[0], 2) for k, v in prof.items()},
        "kernel_launches": {k: v[1] for k, v in prof.items()},
        "roofline": roofline,
        "update_kernels": updates,
        "cpu_baseline": cpu,
        "check": check,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
