"""Race check of stage one's three-stream schedule (CPU model, no GPU).

Stage one splits its work into tasks as in the parallel stage one of the
paper (Section 2.3, the dependency graph of its tasks): generating a panel's
left reflectors (block QRs), applying them to A, B and Q; generating the
right reflectors block by block (each block's factor and its pass over B),
applying them to A and Z.  With the overlapped schedule the library runs the
left passes over Q and A and the right pass over Z on a second stream (only
the right pass over A and the next block QRs wait for the pass over A; during
the QR of B the pass over A runs on the third), and the rows of B above a
bound L (that the next factors do not read) on a third;
L moves down once every `chunk` blocks, and only then does the caller's stream
wait for the far rows.

This test restates, per launch, the entries (rectangles) of A, B, Q, Z and of
the reflector buffers that the launch reads and writes, and the event records
and waits between the streams, derives the happens-before order with vector
clocks, and checks that every two launches that touch a common entry, one of
them writing it, are ordered, in the order of the one-stream schedule.  The
caller's own work before and after the call (filling the inputs, reading the
results) is part of the model.
"""
import bisect

import pytest


class Blocks:
    """Geometry of one panel's chain of blocks (0-based rows, inclusive)."""

    def __init__(self, row0, step, bm, nblk, n):
        self.row0, self.step, self.bm, self.nblk, self.n = row0, step, bm, nblk, n

    def r0(self, k):
        return self.row0 + k * self.step

    def r1(self, k):
        return min(self.n, self.row0 + k * self.step + self.bm) - 1


class Model:
    """Launches, records and waits on three streams, in host order."""

    def __init__(self):
        self.ops = []                       # (stream, index in stream, accesses, clock)
        self.last = {"st": None, "far": None, "qz": None}
        self.count = {"st": 0, "far": 0, "qz": 0}
        self.events = {}
        self.waits = []                     # (stream, event) in host order

    def _push(self, s, acc, dep=None):
        self.count[s] += 1
        prev = self.last[s]
        clock = dict(prev[3]) if prev else {"st": 0, "far": 0, "qz": 0}
        clock[s] = self.count[s]
        if dep is not None:
            for t, v in dep[3].items():
                clock[t] = max(clock[t], v)
        op = (s, self.count[s], acc, clock)
        self.last[s] = op
        self.ops.append(op)
        return op

    def launch(self, s, reads=(), writes=()):
        self._push(s, ([tuple(r) for r in reads], [tuple(w) for w in writes]))

    def record(self, ev, s):
        self.events[ev] = self._push(s, ([], []))

    def wait(self, s, ev):
        self.waits.append((s, ev))
        self._push(s, ([], []), dep=self.events[ev])


def stage_one_schedule(n, nb, p, overlap, chunk=8, with_q=True, with_z=True, skip=()):
    """The host schedule of one stage-one call; `skip` names waits to leave out
    (to check that the model notices)."""
    m = Model()
    bm = p * nb
    ALL = lambda mat: (mat, 0, n - 1, 0, n - 1)
    m.launch("st", writes=[ALL(x) for x in "ABQZ"])            # the caller fills the inputs
    st = "st"
    rec = {"far": False, "lq": False, "rz": False, "fa": False}
    qs = "qz" if overlap else st

    def rows_of(bl):
        return bl.r0(0), bl.r1(bl.nblk - 1)

    def left_phase(X, A2, B2, bl, c0, nc, a2first, b2first, from_block, qr_of_b):
        if rec["lq"] and "lq" not in skip:
            m.wait(st, "lq")
        if rec["fa"]:
            if "fa" not in skip:
                m.wait(st, "fa")
            rec["fa"] = False
        ra, rb = rows_of(bl)
        m.launch(st, reads=[(X, ra, rb, c0, c0 + nc - 1)], writes=[(X, ra, rb, c0, c0 + nc - 1), ("VL", 0, 0, 0, 0)])
        has_a = a2first <= n - 1
        # the pass over A: on `far` during the QR of B (idle then), else on `qz`
        sa = ("far" if qr_of_b else "qz") if overlap else st
        if overlap and (with_q or has_a):
            m.record("gl", st)
        if with_q:
            if overlap and "q_start" not in skip:
                m.wait("qz", "gl")
            cells = ("Q", 0, n - 1, ra, rb)
            m.launch(qs, reads=[cells, ("VL", 0, 0, 0, 0)], writes=[cells])
        if has_a:
            if overlap and "a_start" not in skip:
                m.wait(sa, "gl")
            cells = (A2, ra, rb, a2first, n - 1)
            m.launch(sa, reads=[cells, ("VL", 0, 0, 0, 0)], writes=[cells])
        if overlap and (with_q or (has_a and sa == "qz")):
            m.record("lq", "qz")
            rec["lq"] = True
        if overlap and has_a and sa == "far":
            m.record("fa", "far")
            rec["fa"] = True
        if b2first <= n - 1:
            if rec["far"] and "far_lb" not in skip:
                m.wait(st, "far_done")
            cells = [(B2, bl.r0(k), bl.r1(k), max(b2first, bl.r0(k)) if from_block else b2first, n - 1)
                     for k in range(bl.nblk)]
            m.launch(st, reads=cells + [("VL", 0, 0, 0, 0)], writes=cells)

    def right_phase(bl):
        if rec["rz"] and "rz" not in skip:
            m.wait(st, "rz")
        lprev = -1
        for k in range(bl.nblk - 1, -1, -1):
            r0, r1 = bl.r0(k), bl.r1(k)
            m.launch(st, reads=[("B", r0, r1, r0, r1)], writes=[("VR", k, k, 0, 0)])
            kc = (k // chunk) * chunk
            L = bl.r0(kc - 1 if kc > 0 else 0) if overlap else 0
            assert L <= r0 and (k == 0 or L <= bl.r0(k - 1))
            if overlap:
                m.record("fac", st)
                if 0 <= lprev and L < lprev and "bound" not in skip:
                    m.wait(st, "far_done")
            if r1 >= L:
                cells = ("B", L, r1, r0, r1)
                m.launch(st, reads=[cells, ("VR", k, k, 0, 0)], writes=[cells])
            nr = min(r1 - r0 + 1, nb)
            m.launch(st, writes=[("B", r0, r1, r0, r0 + nr - 1)])
            if overlap and L > 0:
                if "far_start" not in skip:
                    m.wait("far", "fac")
                cells = ("B", 0, L - 1, r0, r1)
                m.launch("far", reads=[cells, ("VR", k, k, 0, 0)], writes=[cells])
                m.record("far_done", "far")
                rec["far"] = True
            lprev = L
        ra, rb = rows_of(bl)
        vr = ("VR", 0, bl.nblk - 1, 0, 0)
        if with_z:
            if overlap:
                m.record("gr", st)
                if "z_start" not in skip:
                    m.wait("qz", "gr")
            m.launch(qs, reads=[("Z", 0, n - 1, ra, rb), vr], writes=[("Z", 0, n - 1, ra, rb)])
            if overlap:
                m.record("rz", "qz")
                rec["rz"] = True
        if rec["lq"] and "la" not in skip:
            m.wait(st, "lq")
        m.launch(st, reads=[("A", 0, n - 1, ra, rb), vr], writes=[("A", 0, n - 1, ra, rb)])

    c0 = 0
    while c0 + 1 < n:                                          # QR of B
        nc = min(nb, n - c0)
        rows = n - c0
        nblk = 1 if rows <= bm else 1 + (rows - bm + (p - 1) * nb - 1) // ((p - 1) * nb)
        left_phase("B", "A", "B", Blocks(c0, (p - 1) * nb, bm, nblk, n), c0, nc, 0, c0 + nc, False, True)
        c0 += nb
    j = 1
    while j <= n - 2:                                          # panels
        j2 = min(n, j + nb - 1)
        num = n - nb - j + 1
        if num <= 0:
            break
        nblk = (num + (p - 1) * nb - 1) // ((p - 1) * nb)
        bl = Blocks(j + nb - 1, (p - 1) * nb, bm, nblk, n)
        left_phase("A", "A", "B", bl, j - 1, j2 - j + 1, j2, bl.r0(0), True, False)
        right_phase(bl)
        j += nb
    if overlap and "join" not in skip:
        m.record("far_done", "far")
        m.wait(st, "far_done")
        m.record("rz", "qz")
        m.wait(st, "rz")
    m.launch(st, writes=[ALL("A"), ALL("B")])                  # exact zeros of the pattern
    m.launch(st, reads=[ALL(x) for x in "ABQZ"])               # the caller reads the results
    return m


def _overlap(a, b):
    return a[0] == b[0] and a[1] <= b[2] and b[1] <= a[2] and a[3] <= b[4] and b[3] <= a[4]


def _conflict(x, y):
    (rx, wx), (ry, wy) = x, y
    return any(_overlap(w, o) for w in wx for o in ry + wy) or any(_overlap(w, o) for w in wy for o in rx)


def races(m):
    """Pairs of launches on different streams that conflict and are unordered."""
    by_stream = {s: [op for op in m.ops if op[0] == s] for s in ("st", "far", "qz")}
    known = {s: [op[3] for op in by_stream[s]] for s in by_stream}
    bad = []
    for b in m.ops:
        sb, ib, accb, vb = b
        if not (accb[0] or accb[1]):
            continue
        for s, lst in by_stream.items():
            if s == sb:
                continue
            # ops on s unknown to b: index > vb[s]; ops on s that do not know b:
            # a prefix of the stream (what a stream knows of sb only grows)
            hi = bisect.bisect_left([c[sb] for c in known[s]], ib)
            for a in lst[vb[s]:hi]:
                if (a[2][0] or a[2][1]) and _conflict(a[2], accb):
                    bad.append((a[0], a[1], sb, ib))
    return bad


@pytest.mark.parametrize("n,nb,p,chunk", [(160, 4, 3, 8), (97, 3, 2, 8), (130, 5, 4, 8), (120, 4, 4, 1),
                                          (150, 2, 8, 3), (64, 16, 4, 8), (2, 1, 2, 8), (41, 16, 4, 8)])
def test_overlapped_schedule_has_no_race(n, nb, p, chunk):
    m = stage_one_schedule(n, nb, p, overlap=True, chunk=chunk)
    assert races(m) == []
    assert m.count["far"] > 0 or n < 3


@pytest.mark.parametrize("with_q,with_z", [(False, True), (True, False), (False, False)])
def test_overlapped_schedule_without_q_or_z(with_q, with_z):
    assert races(stage_one_schedule(120, 4, 3, overlap=True, with_q=with_q, with_z=with_z)) == []


def test_one_stream_schedule_is_trivially_ordered():
    m = stage_one_schedule(100, 4, 3, overlap=False)
    assert m.count["far"] == 0 and m.count["qz"] == 0 and races(m) == []


@pytest.mark.parametrize("wait", ["bound", "lq", "rz", "far_lb", "join", "far_start", "z_start", "q_start", "la", "fa", "a_start"])
def test_model_detects_each_missing_wait(wait):
    """Every wait of the schedule is needed: without any one of them some
    launch races with another."""
    m = stage_one_schedule(160, 4, 3, overlap=True, chunk=2, skip=(wait,))
    assert races(m), wait


def test_the_bound_moves_once_per_chunk():
    """The caller's stream waits for the far rows once per chunk of blocks
    (plus the join and the pass over B of each panel), not once per block."""
    n, nb, p = 400, 4, 3
    m = stage_one_schedule(n, nb, p, overlap=True, chunk=8)
    waits = m.waits.count(("st", "far_done"))
    blocks = sum(1 for op in m.ops if op[0] == "far" and op[2][1])
    panels = len([1 for j in range(1, n - 1, nb) if n - nb - j + 1 > 0])
    assert blocks > 8 * panels and waits < blocks / 4


def test_model_uses_the_library_chunk_length():
    """The model's default chunk is the one the library compiles in."""
    import inspect
    import re
    from pathlib import Path
    src = (Path(__file__).resolve().parents[1] / "paper_2301_07964_amd" / "csrc" / "ht_stage1.hip").read_text()
    m = re.search(r"constexpr int64_t kS1Chunk = (\d+);", src)
    assert m, "kS1Chunk not found"
    default = inspect.signature(stage_one_schedule).parameters["chunk"].default
    assert int(m.group(1)) == default


def test_overlapped_schedule_has_no_race_over_a_grid_of_shapes():
    """A grid of small shapes (n up to 41, panel widths 1..9, p 2..5, chunk
    lengths 1, 3 and the library's), including panels with a single block and
    the last panels' ragged blocks."""
    count = 0
    for n in (3, 4, 7, 12, 19, 28, 41):
        for nb in (1, 2, 3, 5, 9):
            if nb > n - 1:
                continue
            for p in (2, 3, 5):
                for chunk in (1, 3, 8):
                    assert races(stage_one_schedule(n, nb, p, overlap=True, chunk=chunk)) == [], (n, nb, p, chunk)
                    count += 1
    assert count > 250
