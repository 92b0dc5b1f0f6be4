"""GPU tests of the batched stage two (ht_stage2_batched, one persistent
launch over many pencils of uneven n and r), through the C ABI: parity with
the CPU oracle on a sample of pencils, agreement with the single-pencil
ht_stage2, and the invariants of the output contract on the batched workload
distribution (n uniform on [32, 512], r in {4, 8, 16} with r < n/4)."""
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


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _device_pencils(pencils, accumulate=True):
    ht = _ht()
    out = []
    for H, T, r in pencils:
        n = H.shape[0]
        Hd, Td = ht.colmajor(H), ht.colmajor(T)
        Qd = ht.colmajor(np.eye(n, dtype=H.dtype)) if accumulate else None
        Zd = ht.colmajor(np.eye(n, dtype=H.dtype)) if accumulate else None
        out.append((Hd, Td, Qd, Zd, r))
    return out


def _run_batched(pencils, accumulate=True):
    ht = _ht()
    dev = _device_pencils(pencils, accumulate)
    ht.stage2_batched(dev)
    torch.cuda.synchronize()
    return [[ht.to_numpy(x) if x is not None else None for x in p[:4]] for p in dev]


def _sample(count, seed, cplx=False, nhi=512):
    cfg = inputs.batch_configs(count, seed, nhi=nhi)
    out = []
    for b, (n, r) in enumerate(cfg):
        if cplx:
            H, T = inputs.rht_pencil_complex(n, r, seed * 100003 + b)
        else:
            H, T = inputs.rht_pencil(n, r, seed * 100003 + b)
        out.append((H, T, r))
    return out


def test_batched_parity_with_oracle():
    from oracle import oracle as O
    pencils = _sample(24, 1, nhi=200)
    print(f"[batched] parity on {len(pencils)} pencils, n={[p[0].shape[0] for p in pencils]}", flush=True)
    got = _run_batched(pencils)
    for (H, T, r), g in zip(pencils, got):
        ref = O.stage2(H, T, r)
        errs = [rel(a, b) for a, b in zip(g, ref[:4])]
        assert max(errs) <= TOL, (H.shape[0], r, errs)
        assert np.all(np.tril(g[0], -2) == 0) and np.all(np.tril(g[1], -1) == 0)


def test_batched_complex_parity():
    from oracle import oracle as O
    pencils = _sample(6, 2, cplx=True, nhi=120)
    got = _run_batched(pencils)
    for (H, T, r), g in zip(pencils, got):
        ref = O.stage2(H, T, r)
        errs = [rel(a, b) for a, b in zip(g, ref[:4])]
        assert max(errs) <= TOL, (H.shape[0], r, errs)


def test_batched_matches_single_pencil_path():
    ht = _ht()
    pencils = _sample(8, 3, nhi=300)
    got = _run_batched(pencils)
    for (H, T, r), g in zip(pencils, got):
        n = H.shape[0]
        Hd, Td = ht.colmajor(H), ht.colmajor(T)
        Qd, Zd = ht.colmajor(np.eye(n)), ht.colmajor(np.eye(n))
        ht.stage2(Hd, Td, r, Qd, Zd)
        torch.cuda.synchronize()
        single = [ht.to_numpy(x) for x in (Hd, Td, Qd, Zd)]
        errs = [rel(a, b) for a, b in zip(g, single)]
        assert max(errs) <= TOL, (n, r, errs)


def test_batched_edge_cases_and_null_factors():
    rng = np.random.default_rng(5)
    pencils = []
    for n, r in [(0, 2), (1, 3), (2, 4), (3, 1), (5, 4), (40, 31), (33, 8), (20, 40)]:
        H, T = inputs.rht_pencil(n, max(1, min(r, max(n - 1, 1))), int(rng.integers(1 << 30)))
        pencils.append((H, T, r))
    from oracle import oracle as O
    got = _run_batched(pencils, accumulate=False)
    for (H, T, r), g in zip(pencils, got):
        ref = O.stage2(H, T, r, accumulate=False)
        for a, b in zip(g[:2], ref[:2]):
            assert rel(a, b) <= TOL


def test_batched_invariants_full_distribution():
    """256 pencils of the batched workload: exact zeros, orthogonality and
    backward error within 100 n eps for every pencil (computed on the GPU)."""
    ht = _ht()
    cfg = inputs.batch_configs(256, 0)
    dev, orig = [], []
    for b, (n, r) in enumerate(cfg):
        H, T = inputs.rht_pencil(n, r, b)
        Hd, Td = ht.colmajor(H), ht.colmajor(T)
        orig.append((Hd.clone(), Td.clone()))
        I = torch.eye(n, dtype=torch.float64, device="cuda").t()
        dev.append((Hd, Td, I.clone(), I.clone(), r))
    print(f"[batched] 256 pencils, n in [{min(c[0] for c in cfg)}, {max(c[0] for c in cfg)}]", flush=True)
    ht.stage2_batched(dev)
    torch.cuda.synchronize()
    worst = 0.0
    for (Hd, Td, Qd, Zd, r), (H0, T0) in zip(dev, orig):
        n = Hd.shape[0]
        I = torch.eye(n, dtype=torch.float64, device="cuda")
        assert (torch.tril(Hd, -2) == 0).all() and (torch.tril(Td, -1) == 0).all()
        vals = [torch.linalg.norm(Qd.t() @ Qd - I).item(), torch.linalg.norm(Zd.t() @ Zd - I).item(),
                (torch.linalg.norm(Qd @ Hd @ Zd.t() - H0) / torch.linalg.norm(H0)).item(),
                (torch.linalg.norm(Qd @ Td @ Zd.t() - T0) / torch.linalg.norm(T0)).item()]
        assert max(vals) <= 100 * n * EPS, (n, r, vals)
        worst = max(worst, max(vals) / (n * EPS))
    print(f"[batched] worst error / (n eps) = {worst:.3f}", flush=True)


def test_batched_invalid_arguments():
    ht = _ht()
    H = ht.colmajor(np.eye(8))
    with pytest.raises(ht.HTError) as e:
        ht.stage2_batched([(H, H.clone(), None, None, 0)])
    assert e.value.code == -7
    H40 = ht.colmajor(np.eye(40))
    with pytest.raises(ht.HTError) as e:                 # min(r, n-1) = 34 > 32
        ht.stage2_batched([(H40, H40.clone(), None, None, 34)])
    assert e.value.code == 4


def test_back_to_back_batches_on_one_stream():
    """Two batched calls enqueued on one stream without a host synchronisation
    in between (the second reuses the stream's pinned descriptor buffer while
    the first may still run) give the same results as the calls made apart."""
    ht = _ht()
    a = _sample(40, 21)
    b = _sample(17, 22)
    ref_a = _run_batched(a)
    ref_b = _run_batched(b)
    st = torch.cuda.Stream()
    da, db = _device_pencils(a), _device_pencils(b)
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        ht.stage2_batched(da, stream=st)
        ht.stage2_batched(db, stream=st)
    st.synchronize()
    for dev, ref in ((da, ref_a), (db, ref_b)):
        for p, r in zip(dev, ref):
            for x, y in zip(p[:4], r):
                assert np.array_equal(ht.to_numpy(x), y)


def test_reserved_workspace_serves_later_calls():
    """ht_reserve_workspace sizes a stream's workspace once; stage-two and
    stage-one calls on that stream then run (and match the default stream's
    results bit for bit)."""
    ht = _ht()
    n, r = 300, 16
    st = torch.cuda.Stream()
    need = max(ht.workspace_bytes(n, r, 0, True), ht.rhess_workspace_bytes(n, r, 0, True))
    ht.reserve_workspace(need, st)
    H, T = inputs.rht_pencil_complex(n, r, 5)
    outs = []
    for stream in (st, None):
        Hd, Td = ht.colmajor(H), ht.colmajor(T)
        Qd = ht.colmajor(np.eye(n, dtype=H.dtype))
        Zd = ht.colmajor(np.eye(n, dtype=H.dtype))
        torch.cuda.synchronize()
        if stream is None:
            ht.stage2(Hd, Td, r, Qd, Zd)
        else:
            with torch.cuda.stream(stream):
                ht.stage2(Hd, Td, r, Qd, Zd, stream=stream)
        torch.cuda.synchronize()
        outs.append([ht.to_numpy(x) for x in (Hd, Td, Qd, Zd)])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
    A, B = inputs.dense_pencil(n, seed=6, complex_=True)
    Ad, Bd = ht.colmajor(A), ht.colmajor(B)
    with torch.cuda.stream(st):
        ht.rhess(Ad, Bd, r, stream=st)
    st.synchronize()
    An, Bn = ht.to_numpy(Ad), ht.to_numpy(Bd)
    assert np.all(np.tril(An, -(r + 1)) == 0) and np.all(np.tril(Bn, -1) == 0)
    with pytest.raises(ht.HTError):
        ht.reserve_workspace(-1, st)


@pytest.mark.parametrize("threads", [64, 256])
def test_batched_parity_both_modes_up_to_512(threads):
    """Oracle parity of the batched launch on a sample that covers the whole
    batched workload range (n up to 512, r in {4, 8, 16}), with every pencil
    forced onto one wavefront (64) or one workgroup (256) through the tuning
    table; entry by entry within 1e-9."""
    from oracle import oracle as O
    ht = _ht()
    rng = np.random.default_rng(31)
    pencils = []
    for i, (n, r) in enumerate([(512, 4), (500, 16), (451, 8), (384, 16), (300, 4), (257, 8), (200, 16), (129, 4),
                                (96, 8), (64, 8), (40, 4), (33, 4)]):
        H, T = inputs.rht_pencil(n, r, 700 + i)
        pencils.append((H, T, r))
    old = []
    ht.set_batched_tuning([(100000, 0, threads)])
    try:
        got = _run_batched(pencils)
    finally:
        ht.set_batched_tuning(old)
        ht._apply_batched_table(ht.lib())
    for (H, T, r), g in zip(pencils, got):
        ref = O.stage2(H, T, r)
        errs = [rel(a, b) for a, b in zip(g, ref[:4])]
        print(f"[batched {threads}] n={H.shape[0]} r={r} errs={max(errs):.2e}", flush=True)
        assert max(errs) <= TOL, (threads, H.shape[0], r, errs)
        assert np.all(np.tril(g[0], -2) == 0) and np.all(np.tril(g[1], -1) == 0)


def test_batched_tuning_arguments():
    ht = _ht()
    L = ht.lib()
    import ctypes
    a = (ctypes.c_int64 * 1)(100)
    b = (ctypes.c_int64 * 1)(4)
    c = (ctypes.c_int64 * 1)(128)
    P = ctypes.POINTER(ctypes.c_int64)
    assert L.ht_batched_set_tuning(-1, None, None, None) == -1
    assert L.ht_batched_set_tuning(1, None, None, None) == -2
    assert L.ht_batched_set_tuning(1, ctypes.cast(a, P), ctypes.cast(b, P), ctypes.cast(c, P)) == -4
    ht._apply_batched_table(L)
