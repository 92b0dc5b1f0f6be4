"""Request loop for complex128 Hessenberg-triangular reductions on one GPU.

Requests arrive over time (a trace of arrival times); each asks for the
reduction of one pencil to Hessenberg-triangular form with Q and Z
accumulated: an r-HT pencil (stage two only) or a dense pencil (stage one,
ht_rhess_z, then stage two).  Pencils and their Q, Z stay in device memory.

Two policies on the same trace:

* ``fifo``: one request at a time in arrival order, each reduced by its own
  launches (one pencil per launch sequence) on one stream.
* ``continuous``: continuous batching.  A request is admitted as soon as an
  execution slot and HBM for its footprint (6 n^2 complex entries: H, T, Q,
  Z and the payload synthesis; each slot's library workspace is reserved once
  at start, ``ht_reserve_workspace``) are free; large or
  dense requests each take a stream of their own, so their kernels overlap on
  the device; small r-HT requests that are waiting when the batch slot frees
  up are reduced together in one persistent ``ht_stage2_batched_z`` launch.
  Requests that arrive while others run join at the next free slot.

Each slot's stream (and the auxiliary stream the library pairs with it for Q
and Z) needs a hardware queue of its own for the slots' kernels to overlap:
run with GPU_MAX_HW_QUEUES >= 2 * slots + 1 in the environment (HIP reads it
when it initialises).

Latency = completion (the request's last kernel observed finished) minus
arrival, on the host clock, including queueing.  The payload of a request is
synthesised on the device at admission from its seed (standing in for an
upload), with the distributions of ``inputs`` (real and imaginary parts
N(0,1)/sqrt(2); T diagonal 1 + |z|).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the trace
    n: int
    r: int
    dense: bool
    seed: int
    admitted: float = math.nan
    done: float = math.nan
    result: tuple = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_trace(count: int, rate: float, seed: int = 0, nlo: int = 64, nhi: int = 8192, rs=(8, 16, 32),
               p_dense: float = 0.2):
    """Poisson arrivals at ``rate`` per second; n = round(exp(U(ln nlo, ln nhi)));
    r drawn from ``rs`` until r < n/4; dense with probability ``p_dense``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        n = int(round(math.exp(rng.uniform(math.log(nlo), math.log(nhi)))))
        while True:
            r = int(rng.choice(rs))
            if r < n / 4:
                break
        dense = bool(rng.random() < p_dense)
        out.append(Request(i, t, n, r, dense, int(rng.integers(1 << 31))))
    return out


def footprint(req: Request) -> int:
    """Device bytes a request holds while admitted: H, T, Q, Z and two more
    n x n complex matrices of payload synthesis.  The library workspace is not
    part of it: every execution stream's workspace is reserved once, for the
    largest request, when the engine starts."""
    return 6 * req.n * req.n * 16


def workspace_need(nmax: int, rs=(8, 16, 32)) -> int:
    """Largest library workspace (stage two, or stage one) of a complex
    request with n <= nmax and r in rs."""
    import paper_2301_07964_amd as ht
    need = 0
    for r in rs:
        rr = min(r, max(nmax - 1, 1))
        need = max(need, ht.workspace_bytes(nmax, rr, 0, True), ht.rhess_workspace_bytes(nmax, rr, 0, True))
    return need


def _synthesize(req: Request, device):
    """H, T (or A, B for a dense request), Q = Z = I, column-major complex128."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(req.seed)
    n = req.n
    s = 1.0 / math.sqrt(2.0)

    def cn(shape):
        re = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
        im = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
        return torch.complex(re * s, im * s)

    A = cn((n, n))
    B = cn((n, n))
    if not req.dense:
        i = torch.arange(n, device=device)
        A = torch.where(i[:, None] <= i[None, :] + req.r, A, torch.zeros((), dtype=A.dtype, device=device))
        d = 1.0 + cn((n,)).abs()
        B = torch.triu(B, 1) + torch.diag(d.to(torch.complex128))
    out = []
    for X in (A, B, torch.eye(n, dtype=torch.complex128, device=device),
              torch.eye(n, dtype=torch.complex128, device=device)):
        Y = torch.empty_strided((n, n), (1, max(1, n)), dtype=torch.complex128, device=device)
        Y.copy_(X)
        out.append(Y)
    return out


class Engine:
    def __init__(self, policy: str = "continuous", slots: int = 6, budget_bytes: int | None = None,
                 small_n: int = 512, batch_cap: int = 256, keep_results: bool = False, nmax: int = 8192,
                 rs=(8, 16, 32)):
        import torch
        import paper_2301_07964_amd as ht
        assert policy in ("continuous", "fifo")
        self.policy = policy
        self.slots = 1 if policy == "fifo" else slots
        self.small_n = small_n if policy == "continuous" else 0
        self.batch_cap = batch_cap
        self.keep = keep_results
        self.dev = torch.device("cuda:0")
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(self.slots)]
        self.batch_stream = torch.cuda.Stream(device=self.dev)
        # workspaces sized once for the largest request: no allocation (and no
        # synchronisation) inside the loop
        ws = workspace_need(nmax, rs)
        for st in self.streams:
            ht.reserve_workspace(ws, st)
        ht.reserve_workspace(1 << 20, self.batch_stream)       # descriptors of up to ~8k pencils
        torch.cuda.synchronize()
        self.workspace_bytes = ws * len(self.streams)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = budget_bytes
        self.peak_bytes = 0
        self.max_inflight = 0

    # one request (or a batch) on a stream; returns the completion event
    def _launch_single(self, req, stream):
        import torch
        import paper_2301_07964_amd as ht
        with torch.cuda.stream(stream):
            A, B, Q, Z = _synthesize(req, self.dev)
            if req.dense:
                ht.rhess(A, B, req.r, Q, Z, stream=stream)
            ht.stage2(A, B, req.r, Q, Z, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, (A, B, Q, Z)

    def _launch_batch(self, reqs, stream):
        import torch
        import paper_2301_07964_amd as ht
        with torch.cuda.stream(stream):
            mats = [_synthesize(q, self.dev) for q in reqs]
            ht.stage2_batched([(m[0], m[1], m[2], m[3], q.r) for m, q in zip(mats, reqs)], stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, mats

    def run(self, trace, time_limit: float = 1e9, progress=None):
        """Replays ``trace`` in real time; fills admitted/done of every request.
        ``progress(done_count, total, now)`` is called after each completion."""
        pending = sorted(trace, key=lambda q: q.arrival)
        queue = []
        inflight = []               # (event, [reqs], bytes, slot index or -1 for the batch slot, payload)
        free_slots = list(range(self.slots))
        batch_free = self.small_n > 0
        used = 0
        t0 = time.perf_counter()
        pi = 0
        ndone = 0
        while pi < len(pending) or queue or inflight:
            now = time.perf_counter() - t0
            if now > time_limit:
                raise TimeoutError("serving run exceeded its time limit")
            while pi < len(pending) and pending[pi].arrival <= now:
                queue.append(pending[pi])
                pi += 1
            # completions
            still = []
            for ev, reqs, nbytes, slot, payload in inflight:
                if ev.query():
                    tdone = time.perf_counter() - t0
                    for k, q in enumerate(reqs):
                        q.done = tdone
                        if self.keep:
                            q.result = payload[k] if slot < 0 else payload
                    used -= nbytes
                    ndone += len(reqs)
                    if progress is not None:
                        progress(ndone, len(pending), tdone)
                    if slot >= 0:
                        free_slots.append(slot)
                    else:
                        batch_free = True
                else:
                    still.append((ev, reqs, nbytes, slot, payload))
            inflight = still
            # admission
            launched = False
            if batch_free:
                small = [q for q in queue if not q.dense and q.n <= self.small_n]
                take, nbytes = [], 0
                for q in small:
                    f = footprint(q)
                    if len(take) < self.batch_cap and used + nbytes + f <= self.budget:
                        take.append(q)
                        nbytes += f
                if take:
                    tnow = time.perf_counter() - t0
                    for q in take:
                        q.admitted = tnow
                        queue.remove(q)
                    ev, payload = self._launch_batch(take, self.batch_stream)
                    used += nbytes
                    inflight.append((ev, take, nbytes, -1, payload))
                    batch_free = False
                    launched = True
            while free_slots:
                cand = None
                for q in queue:               # arrival order among the requests a slot serves
                    if self.small_n > 0 and not q.dense and q.n <= self.small_n:
                        continue
                    cand = q
                    break
                if cand is None:
                    break
                f = footprint(cand)
                if used + f > self.budget and inflight:
                    break                     # wait for memory (never starve an empty device)
                slot = free_slots.pop(0)
                cand.admitted = time.perf_counter() - t0
                queue.remove(cand)
                ev, payload = self._launch_single(cand, self.streams[slot])
                used += f
                inflight.append((ev, [cand], f, slot, payload))
                launched = True
            self.peak_bytes = max(self.peak_bytes, used)
            self.max_inflight = max(self.max_inflight, sum(len(x[1]) for x in inflight))
            if not launched:
                time.sleep(0.0002)
        import torch
        torch.cuda.synchronize()
        return trace


def summary(trace, wall: float | None = None):
    lat = np.array([q.latency for q in trace])
    end = max(q.done for q in trace)
    start = min(q.arrival for q in trace)
    span = wall if wall is not None else end - start
    return {"requests": len(trace), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2), "mean_ms": round(float(lat.mean()) * 1e3, 2),
            "pencils_per_s": round(len(trace) / span, 3), "span_s": round(span, 3)}
