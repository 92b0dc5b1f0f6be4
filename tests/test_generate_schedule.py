"""Race check of the generation phase's schedule (CPU model, no GPU).

The generation kernel runs one workgroup per sweep of a group (the step
chain) and two helper workgroups per sweep (the far rows of each step's eager
right update, Section 3.2: one for the rows of H, one for those of T).  Step k
of sweep w waits until sweep w-1 has finished its steps up to k+2 and both its
helpers the far rows up to step k+1; each helper of sweep w runs step k once
the sweep's own step k is done.

This test restates, per task, the entries of H and T (and the reflector
records) that the kernel reads and writes, derives the happens-before order
that the waits give, and checks that every two tasks touching a common entry,
one of them writing it, are ordered, and ordered as the unblocked algorithm
orders them (sweep after sweep, step after step).  An entry two unordered
tasks touch would be a data race on the GPU.
"""
import itertools

import pytest


def nblocks(n, r, j):
    """Blocks of sweep j with at least two rows (the unblocked algorithm's count)."""
    return 0 if n - j - 2 < 0 else 1 + (n - j - 2) // r


def rect(mat, r0, r1, c0, c1):
    """Entries (1-based, inclusive ranges) of matrix mat."""
    return {(mat, i, c) for i in range(r0, r1 + 1) for c in range(c0, c1 + 1)}


def tasks_of_group(n, r, j1, j2):
    """{task: (reads, writes)} for the chain ('c', w, k) and the helper tasks
    ('hH', w, k) (far rows of H) and ('hT', w, k) (far rows of T)."""
    kext = nblocks(n, r, j1) + 1
    out = {}
    for w in range(j2 - j1 + 1):
        j = j1 + w
        d = j2 - j
        nbj = nblocks(n, r, j)
        for k in range(kext):
            jb = j + max(0, (k - 1) * r + 1)
            i1 = j + k * r + 1
            i2 = min(j + (k + 1) * r, n)
            i3 = min(j + (k + 2) * r, n)
            rd, wr = set(), set()
            # lazy left updates with the earlier sweeps' reflectors of block k
            if j > j1:
                base, rowmax = j1 + k * r + 1, min(j - 1 + (k + 1) * r, n)
                for mat, col in (("H", jb), ("T", i1 + r - 1)):
                    if col <= n and base <= rowmax:
                        cells = rect(mat, base, rowmax, col, col)
                        rd |= cells
                        wr |= cells
                # the left reflectors (and WY factor columns) of block k of the
                # earlier sweeps; those of block k+1 are staged during step k
                rd |= {(rec, wh, kk) for rec in ("VL", "TF") for wh in range(w) for kk in (k, k + 1) if kk < kext}
            wr |= {("VL", w, k), ("VR", w, k), ("TF", w, k)}
            if k < nbj:
                cells = rect("H", i1, i2, jb, jb)                     # left reflector's column
                rd |= cells
                wr |= cells
                cells = rect("T", i1, i2, i1, i2)                     # T block (left reflector applied)
                rd |= cells
                wr |= cells
                top_h = max(j1 + 1, j1 + 1 + (k + 1 - d) * r)
                near = max(top_h, j1 + (k + 1) * r + 1)
                if near <= i3:
                    cells = rect("H", near, i3, i1, i2)               # near rows of the eager update
                    rd |= cells
                    wr |= cells
            out[("c", w, k)] = (rd, wr)
            rdh, wrh, rdt, wrt = set(), set(), set(), set()
            if k < nbj:
                rdh.add(("VR", w, k))
                rdt.add(("VR", w, k))
                top_h = max(j1 + 1, j1 + 1 + (k + 1 - d) * r)
                near = max(top_h, j1 + (k + 1) * r + 1)
                if top_h <= near - 1:
                    cells = rect("H", top_h, near - 1, i1, i2)
                    rdh |= cells
                    wrh |= cells
                if d >= 1:
                    top_t = max(j1 + 1, j1 + 1 + (k - d) * r)
                    cells = rect("T", top_t, i2, i1, i2)
                    rdt |= cells
                    wrt |= cells
                else:
                    wrt |= rect("T", i1 + 1, i2, i1, i1)              # exact zeros below the diagonal
            out[("hH", w, k)] = (rdh, wrh)
            out[("hT", w, k)] = (rdt, wrt)
    return out, kext


HELPERS = ("hH", "hT")


def edges(q, kext, chain_lag=3, helper_lag=2):
    """Happens-before edges the waits give (each pair: earlier, later)."""
    e = []
    for w in range(q):
        for k in range(kext):
            if k + 1 < kext:
                e.append((("c", w, k), ("c", w, k + 1)))
                for h in HELPERS:
                    e.append(((h, w, k), (h, w, k + 1)))
            for h in HELPERS:
                e.append((("c", w, k), (h, w, k)))
            if w > 0:
                # progress >= k + chain_lag: steps 0 .. k+chain_lag-1 (all of them at the end)
                e.append((("c", w - 1, min(k + chain_lag - 1, kext - 1)), ("c", w, k)))
                for h in HELPERS:
                    e.append(((h, w - 1, min(k + helper_lag - 1, kext - 1)), ("c", w, k)))
    return e


def happens_before(tasks, e):
    succ = {t: [] for t in tasks}
    for a, b in e:
        succ[a].append(b)
    reach = {}

    def dfs(t):
        if t in reach:
            return reach[t]
        s = set()
        for b in succ[t]:
            s.add(b)
            s |= dfs(b)
        reach[t] = s
        return s

    for t in tasks:
        dfs(t)
    return reach


def unblocked_key(t):
    kind, w, k = t
    return (w, k, {"c": 0, "hH": 1, "hT": 2}[kind])


def violations(n, r, q, chain_lag=3, helper_lag=2, j1=1):
    j2 = min(j1 + q - 1, n - 2)
    qq = j2 - j1 + 1
    tasks, kext = tasks_of_group(n, r, j1, j2)
    reach = happens_before(tasks, edges(qq, kext, chain_lag, helper_lag))
    touch = {}
    for t, (rd, wr) in tasks.items():
        for cell in rd | wr:
            touch.setdefault(cell, []).append((t, cell in wr))
    bad = set()
    for cell, lst in touch.items():
        for (a, wa), (b, wb) in itertools.combinations(lst, 2):
            if not (wa or wb):
                continue
            first, second = sorted((a, b), key=unblocked_key)
            if second not in reach[first]:
                bad.add((first, second))
    return bad


@pytest.mark.parametrize("n,r,q", [(40, 3, 4), (61, 4, 4), (70, 4, 2), (90, 8, 8), (75, 5, 3), (50, 2, 6)])
def test_generation_schedule_is_race_free(n, r, q):
    assert violations(n, r, q) == set()


@pytest.mark.parametrize("n,r,q,j1", [(61, 4, 4, 5), (61, 4, 4, 45), (90, 8, 8, 41), (50, 3, 3, 44)])
def test_later_groups_are_race_free(n, r, q, j1):
    # groups further down, including a last group shorter than q
    assert violations(n, r, q, j1=j1) == set()


def block_of(task):
    """Workgroup index of a task's workgroup in the generate kernel's grid:
    sweep w is workgroup 3w, its far-row helpers 3w + 1 (H) and 3w + 2 (T)."""
    kind, w, _ = task
    return 3 * w + {"c": 0, "hH": 1, "hT": 2}[kind]


@pytest.mark.parametrize("q", [1, 2, 5, 8, 32])
def test_every_wait_is_on_a_lower_workgroup(q):
    """Forward progress without co-residency: each wait edge (a task waiting on
    another workgroup's task) points from a lower workgroup index to a higher
    one, so the lowest unfinished workgroup never waits on an undispatched one
    (workgroups are dispatched in index order)."""
    for a, b in edges(q, 6):
        if block_of(a) != block_of(b):
            assert block_of(a) < block_of(b), (a, b)


def test_model_detects_a_missing_wait():
    # waiting for the predecessor's far rows only up to step k (one step too
    # few) leaves its step k+1 far rows unordered with this step's T block
    assert violations(61, 4, 4, helper_lag=1)
    # and a chain stagger of two leaves the predecessor's step k+2 unordered
    assert violations(61, 4, 4, chain_lag=2)


# ------------------------------------------------------------- lookahead

def lookahead_violations(n, r, q, j1=1, tw=16, ahead=1):
    """With lookahead the scratch band of a group is written tile by tile (tw
    columns each) by the previous group's left pass, while this group's
    generation runs.  The first sweep's step k waits until the tiles of
    columns j1 .. min(j1+(k+ahead)r, n) are written (the kernel: ahead = 1).
    Returns the (tile, task) pairs where a task touches a column of H or T
    before that column's tile is ordered before it."""
    j2 = min(j1 + q - 1, n - 2)
    qq = j2 - j1 + 1
    tasks, kext = tasks_of_group(n, r, j1, j2)
    e = edges(qq, kext)
    ntiles = (n + tw - 1) // tw
    alltasks = dict(tasks)
    for t in range(ntiles):
        alltasks[("L", t, 0)] = (set(), set())
    for k in range(kext):
        tneed = (min(j1 + (k + ahead) * r, n) - 1) // tw
        for t in range((j1 - 1) // tw, tneed + 1):
            e.append((("L", t, 0), ("c", 0, k)))
    reach = happens_before(alltasks, e)
    bad = set()
    for task, (rd, wr) in tasks.items():
        for mat, _, c in rd | wr:
            if mat in ("H", "T"):
                tile = ("L", (c - 1) // tw, 0)
                if task not in reach[tile]:
                    bad.add((tile, task))
    return bad


@pytest.mark.parametrize("n,r,q,j1", [(61, 4, 4, 1), (61, 4, 4, 9), (90, 8, 8, 17), (75, 5, 3, 4), (70, 16, 16, 1),
                                      (50, 3, 3, 44)])
@pytest.mark.parametrize("tw", [1, 3, 16])
def test_lookahead_tiles_cover_every_access(n, r, q, j1, tw):
    """Every entry of the scratch band that any task of the group reads or
    writes lies in a tile that the first sweep waited for before a step that
    happens before that task (later sweeps and helpers inherit the order
    through their own waits)."""
    assert lookahead_violations(n, r, q, j1, tw) == set()


def test_lookahead_model_detects_a_short_wait():
    # waiting only for the columns of the steps before k misses step k's block
    assert lookahead_violations(61, 4, 4, tw=1, ahead=0)
