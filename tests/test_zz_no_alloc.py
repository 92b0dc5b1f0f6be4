"""ht_stage2_noalloc (the entry point for callers that cannot allocate: its
workspace is the library's fixed device scratch) against ht_stage2 on the same
inputs, through the C ABI: two calls in a row, the second on a smaller pencil
(the scratch keeps the first call's contents), each within 1e-9 relative
Frobenius and entry-wise of ht_stage2 (the kernels and reflectors are the same,
so in practice the results are equal), plus the size limit and the status
word."""
import ctypes

import numpy as np
import pytest

from paper_2301_07964_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-9


def _ht():
    import paper_2301_07964_amd as ht
    return ht


def _run(H, T, r, noalloc, status=None):
    ht = _ht()
    n = H.shape[0]
    Hd, Td = ht.colmajor(H), ht.colmajor(T)
    Qd = ht.colmajor(np.eye(n))
    Zd = ht.colmajor(np.eye(n))
    if noalloc:
        ht.stage2_noalloc(Hd, Td, r, Qd, Zd, status=status)
    else:
        ht.stage2(Hd, Td, r, Qd, Zd)
    torch.cuda.synchronize()
    return [ht.to_numpy(x) for x in (Hd, Td, Qd, Zd)]


def _close(a, b):
    for x, y in zip(a, b):
        ny = np.linalg.norm(y)
        assert np.linalg.norm(x - y) <= TOL * ny
        assert np.max(np.abs(x - y)) <= TOL * np.max(np.abs(y))


def test_noalloc_matches_stage2_twice_then_smaller():
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    for n, r, seed in ((1500, 32, 0), (700, 16, 1)):
        print(f"[noalloc] n={n} r={r} seed={seed}", flush=True)
        H, T = inputs.rht_pencil(n, r, seed)
        ref = _run(H, T, r, noalloc=False)
        got = _run(H, T, r, noalloc=True, status=status)
        _close(got, ref)
        assert int(status.item()) == 0
        assert np.all(np.tril(got[0], -2) == 0) and np.all(np.tril(got[1], -1) == 0)


def test_noalloc_size_limit_and_arguments():
    ht = _ht()
    L = ht.lib()
    # a size whose workspace exceeds the scratch is rejected before any work
    n, r = 6000, 32
    assert ht.workspace_bytes(n, r) > ht.NOALLOC_SCRATCH_BYTES
    H = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(H.data_ptr())
    assert L.ht_stage2_noalloc(p, p, None, None, n, r, n, None, None) == 6      # HT_ERR_SCRATCH
    assert L.ht_stage2_noalloc(None, None, None, None, -1, 2, 1, None, None) == -5
    assert L.ht_stage2_noalloc(None, None, None, None, 4, 0, 4, None, None) == -6
    assert L.ht_stage2_noalloc(None, None, None, None, 4, 2, 3, None, None) == -7
    assert L.ht_stage2_noalloc(None, None, None, None, 4, 2, 4, None, None) == -1


def test_noalloc_reports_a_wait_that_gives_up():
    """Failure path forced from the host (wait limit 0: every wait gives up
    without polling, every workgroup exits): the caller's status word gets
    bit 1; with the limit restored the next call matches ht_stage2."""
    ht = _ht()
    n, r = 300, 8
    H, T = inputs.rht_pencil(n, r, 6)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    old = ht.set_knob(ht.KNOB_WAIT_POLLS, 0)
    try:
        _run(H, T, r, noalloc=True, status=status)
    finally:
        ht.set_knob(ht.KNOB_WAIT_POLLS, old)
    assert int(status.item()) & 1
    status.zero_()
    _close(_run(H, T, r, noalloc=True, status=status), _run(H, T, r, noalloc=False))
    assert int(status.item()) == 0
