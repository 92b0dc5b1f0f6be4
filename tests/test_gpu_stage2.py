"""GPU parity of ht_stage2 / ht_stage2_z (C ABI through the Python binding)
against the CPU oracle (unblocked stage two, Section 3.1), plus the invariants
of the output contract.  Tolerance: 1e-9 relative Frobenius norm on each of
H, T, Q and Z (delaying the updates reorders the arithmetic, not the
reflectors), and beside it 1e-9 on the largest entry-wise difference relative
to the largest entry, which a localised error cannot hide in."""
import numpy as np
import pytest

from paper_2301_07964_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
TOL = 1e-9


def _ht():
    import paper_2301_07964_amd as ht
    return ht


def run_gpu(H, T, r, q=0, accumulate=True):
    ht = _ht()
    n = H.shape[0]
    Hd, Td = ht.colmajor(H), ht.colmajor(T)
    Qd = Zd = None
    if accumulate:
        Qd = ht.colmajor(np.eye(n, dtype=H.dtype))
        Zd = ht.colmajor(np.eye(n, dtype=H.dtype))
    ht.stage2(Hd, Td, r, Qd, Zd, q=q)
    torch.cuda.synchronize()
    out = [ht.to_numpy(Hd), ht.to_numpy(Td)]
    out += [ht.to_numpy(Qd), ht.to_numpy(Zd)] if accumulate else [None, None]
    return out


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_max(a, b):
    """max |a - b| over the entries, relative to max |b|."""
    mb = np.max(np.abs(b)) if b.size else 0.0
    return (np.max(np.abs(a - b)) if a.size else 0.0) / (mb if mb > 0 else 1.0)


def oracle_threads():
    """Host threads for the oracle (bitwise equal to one thread), at most 16."""
    from oracle import oracle as O
    return max(1, min(16, O.host_cores()))


def check_parity(H, T, r, q=0):
    from oracle import oracle as O
    print(f"[parity] n={H.shape[0]} r={r} q={q} complex={np.iscomplexobj(H)}", flush=True)
    ref = O.stage2(H, T, r)
    got = run_gpu(H, T, r, q)
    errs = [rel(g, o) for g, o in zip(got, ref[:4])]
    assert max(errs) <= TOL, f"relative errors H,T,Q,Z = {errs}"
    emax = [rel_max(g, o) for g, o in zip(got, ref[:4])]
    assert max(emax) <= TOL, f"entry-wise relative errors H,T,Q,Z = {emax}"
    n = H.shape[0]
    # exact zero structure and the first columns of Q, Z
    assert np.all(np.tril(got[0], -2) == 0) and np.all(np.tril(got[1], -1) == 0)
    if n > 0:
        e1 = np.zeros(n)
        e1[0] = 1
        assert np.array_equal(got[2][:, 0], e1) and np.array_equal(got[3][:, 0], e1)
    return errs


@pytest.mark.parametrize("n,r,seed", [(256, 8, 0), (300, 7, 1), (200, 16, 2), (130, 32, 3), (97, 4, 4), (64, 3, 5)])
def test_parity_real(n, r, seed):
    H, T = inputs.rht_pencil(n, r, seed)
    check_parity(H, T, r)


@pytest.mark.parametrize("q", [1, 2, 5, 8])
def test_parity_group_sizes(q):
    H, T = inputs.rht_pencil(181, 8, 10)
    check_parity(H, T, 8, q)


@pytest.mark.parametrize("n,r,seed", [(150, 5, 0), (128, 8, 1), (70, 16, 2), (90, 4, 4), (160, 32, 3), (300, 8, 5)])
def test_parity_complex(n, r, seed):
    H, T = inputs.rht_pencil_complex(n, r, seed)
    check_parity(H, T, r)


@pytest.mark.parametrize("n,r,seed", [(400, 16, 5), (400, 32, 5)])
def test_parity_complex_at_the_sensitivity_floor(n, r, seed):
    """Larger complex pencils of the generator are sensitive: the oracle's own
    output moves by up to ~1e-7 when the band of H is perturbed by 1e-15
    relative, so no implementation can meet 1e-9 there.  The GPU result must
    then lie within 10x of that floor (and within 1e-9 where the floor is
    below 1e-10)."""
    from oracle import oracle as O
    H, T = inputs.rht_pencil_complex(n, r, seed)
    ref = O.stage2(H, T, r)
    rng = np.random.default_rng(1)
    P = rng.standard_normal(H.shape) + 1j * rng.standard_normal(H.shape)
    ref2 = O.stage2(H + 1e-15 * np.abs(H) * P, T, r)
    floor = max(rel(a, b) for a, b in zip(ref2[:4], ref[:4]))
    got = run_gpu(H, T, r)
    errs = [rel(g, o) for g, o in zip(got, ref[:4])]
    print(f"[parity] n={n} r={r} complex: floor {floor:.2e}, errors {errs}", flush=True)
    assert max(errs) <= max(1e-9, 10 * floor), (errs, floor)


@pytest.mark.parametrize("n,r", [(0, 3), (1, 3), (2, 3), (3, 1), (3, 2), (5, 4), (12, 30), (40, 1)])
def test_edge_sizes(n, r):
    H, T = inputs.rht_pencil(n, min(r, max(n - 1, 0)), 3)
    check_parity(H, T, r)


def test_no_accumulation_matches():
    H, T = inputs.rht_pencil(160, 8, 7)
    a = run_gpu(H, T, 8)
    b = run_gpu(H, T, 8, accumulate=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_deterministic():
    H, T = inputs.rht_pencil(333, 16, 8)
    a = run_gpu(H, T, 16)
    b = run_gpu(H, T, 16)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_invalid_arguments():
    ht = _ht()
    n = 8
    H = ht.colmajor(np.eye(n))
    with pytest.raises(ht.HTError) as e:
        ht.stage2(H, H.clone(), 0)
    assert e.value.code == -6
    import ctypes
    assert ht.lib().ht_stage2(None, None, None, None, -1, 2, 1, None) == -5
    assert ht.lib().ht_stage2(None, None, None, None, 4, 2, 2, None) == -7
    assert ht.lib().ht_stage2(None, None, None, None, 4, 2, 4, None) == -1
    assert ht.lib().ht_stage2_q(ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(H.data_ptr()), None, None, 8, 2, 8, 3, None) == -8


@pytest.mark.parametrize("n,r,q", [(1100, 8, 8), (1030, 16, 16), (700, 8, 4), (900, 32, 32)])
def test_parity_many_windows(n, r, q):
    """Regression: more than ~64 windows per group with q = r once amplified
    rounding residue left in structurally-zero entries between groups."""
    H, T = inputs.rht_pencil(n, r, 0)
    check_parity(H, T, r, q)


def _backward(Hin, Tin, r, q=0):
    ht = _ht()
    n = Hin.shape[0]
    H0 = ht.colmajor(Hin)
    T0 = ht.colmajor(Tin)
    Hd, Td = H0.clone(), T0.clone()
    Qd = torch.eye(n, dtype=H0.dtype, device=H0.device).t().contiguous().t()
    Zd = Qd.clone()
    ht.stage2(Hd, Td, r, Qd, Zd, q=q)
    torch.cuda.synchronize()
    I = torch.eye(n, dtype=H0.dtype, device=H0.device)
    res = {
        "orthQ": torch.linalg.norm(Qd.conj().t() @ Qd - I).item(),
        "orthZ": torch.linalg.norm(Zd.conj().t() @ Zd - I).item(),
        "bH": (torch.linalg.norm(Qd @ Hd @ Zd.conj().t() - H0) / torch.linalg.norm(H0)).item(),
        "bT": (torch.linalg.norm(Qd @ Td @ Zd.conj().t() - T0) / torch.linalg.norm(T0)).item(),
        "zeros": bool((torch.tril(Hd, -2) == 0).all().item() and (torch.tril(Td, -1) == 0).all().item()),
    }
    return res


@pytest.mark.parametrize("n,r,cplx", [(2048, 8, False), (4096, 16, False), (3000, 32, False), (2048, 32, True),
                                      (1500, 4, True)])
def test_backward_error_large(n, r, cplx):
    """Invariants at sizes the oracle is too slow for: exact zeros, orthogonality and
    backward error within 100 n eps (eps = 2^-52)."""
    print(f"[backward] n={n} r={r} complex={cplx}", flush=True)
    H, T = (inputs.rht_pencil_complex if cplx else inputs.rht_pencil)(n, r, 1)
    res = _backward(H, T, r)
    bound = 100 * n * EPS
    assert res["zeros"], res
    assert max(res["orthQ"], res["orthZ"], res["bH"], res["bT"]) <= bound, (res, bound)


# ---------------------------------------------------------------- full sizes

def _sweeps_gpu(H, T, r, q, jmax):
    ht = _ht()
    n = H.shape[0]
    Hd, Td = ht.colmajor(H), ht.colmajor(T)
    Qd = torch.eye(n, dtype=Hd.dtype, device=Hd.device).t().contiguous().t()
    Zd = Qd.clone()
    ht.stage2(Hd, Td, r, Qd, Zd, q=q, jmax=jmax)
    torch.cuda.synchronize()
    assert ht.stream_status() == 0
    out = []
    for x in (Hd, Td, Qd, Zd):
        out.append(ht.to_numpy(x))
        del x
    del Hd, Td, Qd, Zd
    torch.cuda.empty_cache()
    return out


def _compare(got, ref, what, floor=(0.0, 0.0)):
    """H, T, Q, Z against the oracle: relative Frobenius error within
    max(1e-9, 10 x floor[0]) and entry-wise error (relative to the largest
    entry) within max(1e-9, 10 x floor[1]), where `floor` is the oracle's own
    response to a rounding-level perturbation of its input (see
    sensitivity_floor)."""
    errs = [rel(g, o) for g, o in zip(got, ref[:4])]
    emax = [rel_max(g, o) for g, o in zip(got, ref[:4])]
    bf, bm = max(TOL, 10 * floor[0]), max(TOL, 10 * floor[1])
    print(f"[parity] {what}: rel H,T,Q,Z = {errs}; entry-wise = {emax}; floor {floor}; bounds {bf:.2e} {bm:.2e}",
          flush=True)
    assert max(errs) <= bf, errs
    assert max(emax) <= bm, emax


def sensitivity_floor(H, T, r, ref, jmax=-1):
    """How far the oracle's own H, T, Q, Z move when the band of H is perturbed
    by 1e-15 relative (a few units of rounding per entry): (max relative
    Frobenius change, max entry-wise change relative to the largest entry).
    Reordering the arithmetic, as the delayed updates do, perturbs at that
    level, so no implementation can be asked to agree more closely."""
    from oracle import oracle as O
    rng = np.random.default_rng(1)
    P = rng.standard_normal(H.shape)
    if np.iscomplexobj(H):
        P = P + 1j * rng.standard_normal(H.shape)
    Hp = H + 1e-15 * np.abs(H) * P
    del P
    ref2 = O.stage2(Hp, T, r, jmax=jmax)
    del Hp
    return (max(rel(a, b) for a, b in zip(ref2[:4], ref[:4])),
            max(rel_max(a, b) for a, b in zip(ref2[:4], ref[:4])))


@pytest.mark.parametrize("n", [8192, 16384])
def test_parity_first_two_groups_at_full_size(n):
    """The headline shapes (r = q = 32, real): the first two groups of sweeps
    (jmax = 64) of the GPU path at n = 8192 and n = 16384 against the oracle's
    first 64 sweeps.  At these sizes the matrix-core right update runs with two
    16-row tiles per wavefront, the variant the full reductions use.

    These pencils are sensitive: a 1e-15 relative perturbation of H's band
    moves the oracle's own result by about 5e-10 (Frobenius) and 8e-9
    (largest entry) at n = 8192, and 5e-9 and 1.3e-7 at n = 16384, where
    near-singular diagonal blocks of T make the direction of the opposite
    reflector ill-determined.  The bound is therefore 10x that floor,
    measured here on the same input, and 1e-9 where the floor is lower."""
    from oracle import oracle as O
    r = q = 32
    jmax = 64
    print(f"[parity] n={n} r={r} q={q} jmax={jmax}: generating", flush=True)
    H, T = inputs.rht_pencil(n, r, 0)
    got = _sweeps_gpu(H, T, r, q, jmax)
    old = O.set_threads(oracle_threads())
    try:
        ref = O.stage2(H, T, r, jmax=jmax)
        floor = sensitivity_floor(H, T, r, ref, jmax)
    finally:
        O.set_threads(old)
    del H, T
    _compare(got, ref, f"n={n} r={r} jmax={jmax}", floor)
    # the structure after 64 sweeps: columns 1..64 of H reduced
    assert np.all(np.tril(got[0][:, :jmax], -2) == 0)


@pytest.mark.parametrize("n,r,seed", [(1000, 32, 0), (1030, 16, 1), (700, 8, 2)])
def test_parity_two_row_tiles(n, r, seed):
    """The matrix-core right update with two 16-row tiles per wavefront (the
    n >= 8192 choice), forced at sizes the full oracle runs in seconds."""
    ht = _ht()
    H, T = inputs.rht_pencil(n, r, seed)
    old = ht.set_knob(ht.KNOB_UPDATE_TILE_ROWS, 2)
    try:
        check_parity(H, T, r)
    finally:
        ht.set_knob(ht.KNOB_UPDATE_TILE_ROWS, old)


def test_parity_full_reduction_n4096_r16():
    """The n = 4096, r = 16 workload reduced completely (Q, Z accumulated),
    against the oracle run on the host cores (bitwise equal to one thread),
    within 10x the oracle's own sensitivity floor (1e-9 where that is lower)."""
    from oracle import oracle as O
    n, r = 4096, 16
    H, T = inputs.rht_pencil(n, r, 0)
    got = _sweeps_gpu(H, T, r, 0, -1)
    old = O.set_threads(oracle_threads())
    try:
        ref = O.stage2(H, T, r)
        floor = sensitivity_floor(H, T, r, ref)
    finally:
        O.set_threads(old)
    _compare(got, ref, f"n={n} r={r} full", floor)
    assert np.all(np.tril(got[0], -2) == 0) and np.all(np.tril(got[1], -1) == 0)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("jmax", [0, 1, 7, 8, 13, 80, 198])
def test_sweeps_prefix(jmax, cplx):
    """ht_stage2_sweeps: the first jmax sweeps (groups of q = 8, the last cut
    at jmax) against the oracle's first jmax sweeps."""
    from oracle import oracle as O
    n, r, q = 200, 8, 8
    H, T = (inputs.rht_pencil_complex if cplx else inputs.rht_pencil)(n, r, 11)
    got = _sweeps_gpu(H, T, r, q, jmax)
    ref = O.stage2(H, T, r, jmax=jmax)
    _compare(got, ref, f"sweeps jmax={jmax} complex={cplx}")
    for g, o in zip(got[:2], ref[:2]):
        assert np.all(g[o == 0] == 0), "an entry the oracle holds at exact zero is nonzero"


def test_wait_give_up_is_reported():
    """Failure path of the generate kernel's bounded waits, forced from the host:
    with a wait limit of 0 every wait gives up without polling, every workgroup
    still exits, and ht_stream_status reports HT_ERR_TIMEOUT once.  With the
    limit restored the next call is correct and the status is clear."""
    ht = _ht()
    n, r = 300, 8
    H, T = inputs.rht_pencil(n, r, 6)
    assert ht.stream_status() == 0
    old = ht.set_knob(ht.KNOB_WAIT_POLLS, 0)
    try:
        Hd, Td = ht.colmajor(H), ht.colmajor(T)
        ht.stage2(Hd, Td, r)
        torch.cuda.synchronize()
    finally:
        ht.set_knob(ht.KNOB_WAIT_POLLS, old)
    assert ht.stream_status() == 5          # HT_ERR_TIMEOUT
    assert ht.stream_status() == 0          # read and cleared
    check_parity(H, T, r)
    assert ht.stream_status() == 0


def test_knob_arguments():
    ht = _ht()
    L = ht.lib()
    assert L.ht_set_knob(0, 1) == -1 and L.ht_get_knob(99) == -1
    assert L.ht_set_knob(ht.KNOB_WAIT_POLLS, -1) == -2
    assert L.ht_set_knob(ht.KNOB_UPDATE_TILE_ROWS, 3) == -2
    assert L.ht_get_knob(ht.KNOB_UPDATE_TILE_ROWS) == 0
    assert L.ht_set_knob(ht.KNOB_LOOKAHEAD, 3) == -2 and L.ht_set_knob(ht.KNOB_LOOKAHEAD, -1) == -2
    assert L.ht_get_knob(ht.KNOB_LOOKAHEAD) == 1


# ------------------------------------------------------------- lookahead

def _with_lookahead(on, fn):
    ht = _ht()
    old = ht.set_knob(ht.KNOB_LOOKAHEAD, 2 if on else 0)      # 2: also below the automatic size limit
    try:
        return fn()
    finally:
        ht.set_knob(ht.KNOB_LOOKAHEAD, old)


@pytest.mark.parametrize("n,r,q,jmax,acc,trw,cplx", [
    (900, 32, 32, -1, True, 0, False), (2100, 32, 32, -1, True, 0, False), (1500, 32, 7, -1, True, 0, False),
    (1200, 32, 32, 70, True, 0, False), (1000, 32, 32, -1, False, 0, False), (33, 32, 32, -1, True, 0, False),
    (4096, 32, 32, 96, True, 0, False), (1000, 16, 16, -1, True, 0, False), (1030, 16, 16, -1, True, 2, False),
    (777, 8, 5, -1, True, 1, False), (1111, 8, 8, -1, True, 2, False), (500, 4, 4, -1, True, 0, False),
    (300, 4, 3, 100, False, 2, False), (700, 32, 32, -1, True, 0, True), (530, 16, 16, -1, True, 0, True),
    (333, 8, 5, -1, True, 0, True), (400, 4, 4, 150, False, 0, True), (700, 32, 11, 90, True, 0, True)])
def test_lookahead_is_bitwise_the_sequential_order(n, r, q, jmax, acc, trw, cplx):
    """Lookahead (Section 3.3; r in {4, 8, 16, 32}): the generation of group
    g+1 runs while the left updates of group g are in progress, reading each
    tile of its scratch band once that tile's epilogue has written it.  Every
    kernel does the same arithmetic on the same values as in the sequential
    order, so the outputs are bitwise equal; real and complex pencils, n not
    a multiple of 16 (and, with two 16-column tiles per wavefront, an odd
    number of tiles), groups cut by jmax, q < r, no accumulation and a
    single group are covered."""
    ht = _ht()
    H, T = (inputs.rht_pencil_complex if cplx else inputs.rht_pencil)(n, r, 17)
    print(f"[lookahead] n={n} r={r} q={q} jmax={jmax} acc={acc} tile rows={trw} complex={cplx}", flush=True)
    old_trw = ht.set_knob(ht.KNOB_UPDATE_TILE_ROWS, trw)

    def run():
        Hd, Td = ht.colmajor(H), ht.colmajor(T)
        Qd = ht.colmajor(np.eye(n, dtype=H.dtype)) if acc else None
        Zd = ht.colmajor(np.eye(n, dtype=H.dtype)) if acc else None
        ht.stage2(Hd, Td, min(r, n - 1), Qd, Zd, q=min(q, n - 1), jmax=jmax)
        torch.cuda.synchronize()
        assert ht.stream_status() == 0
        return [ht.to_numpy(x) for x in (Hd, Td, Qd, Zd) if x is not None]

    try:
        on = _with_lookahead(True, run)
        off = _with_lookahead(False, run)
    finally:
        ht.set_knob(ht.KNOB_UPDATE_TILE_ROWS, old_trw)
    for a, b in zip(on, off):
        assert np.array_equal(a, b)


def test_concurrent_calls_on_several_streams():
    """Four r = 32 reductions enqueued at once on four streams (the serving
    loop's pattern).  A lookahead call's first sweep waits for the same call's
    left pass, and each call's generation takes 3q = 96 whole compute units,
    so only one stream's call at a time may take the lookahead schedule; the
    others run their groups in sequence.  Every result must be bitwise that of
    the sequential order on one stream, and no wait may give up."""
    ht = _ht()
    n, r = 1500, 32
    pencils = [inputs.rht_pencil(n, r, 40 + i) for i in range(4)]
    old = ht.set_knob(ht.KNOB_LOOKAHEAD, 0)
    try:
        ref = []
        for H, T in pencils:
            Hd, Td = ht.colmajor(H), ht.colmajor(T)
            Qd, Zd = ht.colmajor(np.eye(n)), ht.colmajor(np.eye(n))
            ht.stage2(Hd, Td, r, Qd, Zd)
            torch.cuda.synchronize()
            ref.append([ht.to_numpy(x) for x in (Hd, Td, Qd, Zd)])
    finally:
        ht.set_knob(ht.KNOB_LOOKAHEAD, old)
    assert ht.stream_status() == 0
    streams = [torch.cuda.Stream() for _ in pencils]
    outs = []
    for (H, T), st in zip(pencils, streams):
        with torch.cuda.stream(st):
            Hd, Td = ht.colmajor(H), ht.colmajor(T)
            Qd, Zd = ht.colmajor(np.eye(n)), ht.colmajor(np.eye(n))
        st.synchronize()
        outs.append((Hd, Td, Qd, Zd))
    print("[concurrent] enqueueing 4 calls", flush=True)
    # a shorter wait limit (about a quarter of a second of polling): a wait
    # that could not end would show as a timeout in the status, not as a stall
    old_polls = ht.set_knob(ht.KNOB_WAIT_POLLS, 1 << 19)
    try:
        for (Hd, Td, Qd, Zd), st in zip(outs, streams):
            ht.stage2(Hd, Td, r, Qd, Zd, stream=st)
        torch.cuda.synchronize()
    finally:
        ht.set_knob(ht.KNOB_WAIT_POLLS, old_polls)
    for st in streams:
        assert ht.stream_status(st) == 0
    for got, exp in zip(outs, ref):
        for a, b in zip(got, exp):
            assert np.array_equal(ht.to_numpy(a), b)


def test_lookahead_parity_vs_oracle():
    """The lookahead path (the default at r = 32) against the oracle, with a
    group count that leaves a short last group."""
    H, T = inputs.rht_pencil(1111, 32, 23)
    check_parity(H, T, 32)


def test_lookahead_wait_give_up_is_reported():
    """The lookahead wait of the generate phase is bounded like the others:
    with a wait limit of 0 it gives up, every kernel exits, the status word
    reports HT_ERR_TIMEOUT, and the next call is correct."""
    ht = _ht()
    n, r = 700, 32
    H, T = inputs.rht_pencil(n, r, 8)
    assert ht.stream_status() == 0
    old = ht.set_knob(ht.KNOB_WAIT_POLLS, 0)
    old_la = ht.set_knob(ht.KNOB_LOOKAHEAD, 2)              # also below the automatic size limit
    try:
        Hd, Td = ht.colmajor(H), ht.colmajor(T)
        ht.stage2(Hd, Td, r, ht.colmajor(np.eye(n)), ht.colmajor(np.eye(n)))
        torch.cuda.synchronize()
    finally:
        ht.set_knob(ht.KNOB_WAIT_POLLS, old)
        ht.set_knob(ht.KNOB_LOOKAHEAD, old_la)
    assert ht.stream_status() == 5
    assert ht.stream_status() == 0
    check_parity(H, T, r)
    assert ht.stream_status() == 0


# ------------------------------------------------------------- singular T

def _gpu_stage2_from(H, T, r, Q, Z):
    ht = _ht()
    Hd, Td, Qd, Zd = ht.colmajor(H), ht.colmajor(T), ht.colmajor(Q), ht.colmajor(Z)
    ht.stage2(Hd, Td, r, Qd, Zd)
    torch.cuda.synchronize()
    return [ht.to_numpy(x) for x in (Hd, Td, Qd, Zd)]


def _floor_from(H, T, r, Q, Z, ref):
    from oracle import oracle as O
    rng = np.random.default_rng(1)
    P = rng.standard_normal(H.shape)
    if np.iscomplexobj(H):
        P = P + 1j * rng.standard_normal(H.shape)
    ref2 = O.stage2(H + 1e-15 * np.abs(H) * P, T, r, Q=Q, Z=Z)
    return (max(rel(a, b) for a, b in zip(ref2[:4], ref[:4])),
            max(rel_max(a, b) for a, b in zip(ref2[:4], ref[:4])))


@pytest.mark.parametrize("n,r,seed", [(200, 8, 0), (300, 16, 1), (260, 32, 2)])
def test_stage2_saddle_point_vs_oracle(n, r, seed):
    """Saddle-point pencils ([X Y; Y^T 0], [I 0; 0 0]) with a quarter of
    infinite eigenvalues: B is singular, so T and many of the diagonal blocks
    whose RQ gives the opposite reflector are singular too (Section 4's
    saddle-point experiments).  The r-HT input comes from the oracle's stage
    one; the GPU's stage two is compared element by element with the oracle's
    on that same input (the HT form is not unique when T is singular, so the
    two-stage paths are not compared), within max(1e-9, 10 x the oracle's own
    sensitivity floor), and the result keeps rank(T) = rank(B) and the
    backward error towards the original pencil."""
    from oracle import oracle as O
    print(f"[saddle] n={n} r={r} seed={seed}", flush=True)
    A, Bm = inputs.saddle_point_pencil(n, 0.25, seed=seed)
    H0, T0, Q0, Z0, _ = O.rhess(A, Bm, r, 8)
    assert np.linalg.matrix_rank(T0) < n
    ref = O.stage2(H0, T0, r, Q=Q0, Z=Z0)
    got = _gpu_stage2_from(H0, T0, r, Q0, Z0)
    _compare(got, ref, f"saddle n={n} r={r}", _floor_from(H0, T0, r, Q0, Z0, ref))
    H, T, Q, Z = got
    assert np.all(np.tril(H, -2) == 0) and np.all(np.tril(T, -1) == 0)
    bound = 100 * n * EPS
    assert np.linalg.norm(Q @ H @ Z.T - A) / np.linalg.norm(A) <= bound
    assert np.linalg.norm(Q @ T @ Z.T - Bm) / np.linalg.norm(Bm) <= bound
    assert np.linalg.matrix_rank(T) == np.linalg.matrix_rank(Bm)


@pytest.mark.parametrize("n,r,cplx", [(180, 8, False), (240, 16, False), (200, 32, False), (150, 8, True),
                                      (160, 16, True)])
def test_stage2_singular_T_vs_oracle(n, r, cplx):
    """r-HT pencils of the generator with every seventh diagonal entry of T
    set to zero (stage two alone, real and complex): the blocks that contain
    such an entry are singular, and the RQ-based opposite reflector must then
    reproduce the oracle's (its direction is a null vector of the block)."""
    from oracle import oracle as O
    print(f"[singular T] n={n} r={r} complex={cplx}", flush=True)
    H, T = (inputs.rht_pencil_complex if cplx else inputs.rht_pencil)(n, r, 21)
    T = T.copy()
    idx = np.arange(3, n, 7)
    T[idx, idx] = 0
    I = np.eye(n, dtype=H.dtype)
    ref = O.stage2(H, T, r)
    got = _gpu_stage2_from(H, T, r, I, I)
    _compare(got, ref, f"singular T n={n} r={r} complex={cplx}", _floor_from(H, T, r, I, I, ref))
    assert np.all(np.tril(got[0], -2) == 0) and np.all(np.tril(got[1], -1) == 0)
    assert np.linalg.matrix_rank(got[1]) == np.linalg.matrix_rank(T)
