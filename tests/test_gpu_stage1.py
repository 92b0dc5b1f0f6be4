"""GPU tests of stage one (ht_rhess / ht_rhess_z, through the C ABI).

Stage one's r-HT output depends on the blocking, and the GPU factors B with
a blocked (overlapping-block) QR, so it is not compared element-wise with the
oracle.  What the problem fixes is checked instead: the structure (exact
zeros), orthogonality of Q and Z and the backward error (<= 100 n eps), the
first columns of Q and Z, and -- after stage two -- the Hessenberg-triangular
form itself, which is unique once Q e1 is fixed: the full two-stage GPU path
equals the oracle's two-stage path in canonical form (diagonal unimodular
scaling normalised) to 1e-9."""
import numpy as np
import pytest

from paper_2301_07964_amd import inputs
from tests import lapack_ref as LR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _ht():
    import paper_2301_07964_amd as ht
    return ht


def fro(x):
    return float(np.linalg.norm(x))


def _gpu_rhess(A, B, r, p=0, stage2=False):
    ht = _ht()
    n = A.shape[0]
    Ad, Bd = ht.colmajor(A), ht.colmajor(B)
    Qd, Zd = ht.colmajor(np.eye(n, dtype=A.dtype)), ht.colmajor(np.eye(n, dtype=A.dtype))
    ht.rhess(Ad, Bd, r, Qd, Zd, p=p)
    if stage2:
        ht.stage2(Ad, Bd, r, Qd, Zd)
    torch.cuda.synchronize()
    return [ht.to_numpy(x) for x in (Ad, Bd, Qd, Zd)]


def _check_invariants(A, B, Ao, Bo, Q, Z, r):
    n = A.shape[0]
    rr = min(r, max(n - 1, 1))
    assert np.all(np.tril(Ao, -(rr + 1)) == 0) and np.all(np.tril(Bo, -1) == 0)
    I = np.eye(n)
    bound = 100 * n * EPS
    vals = [fro(Q.conj().T @ Q - I), fro(Z.conj().T @ Z - I),
            fro(Q @ Ao @ Z.conj().T - A) / fro(A), fro(Q @ Bo @ Z.conj().T - B) / fro(B)]
    assert max(vals) <= bound, (vals, bound)
    return vals


@pytest.mark.parametrize("n,r,p,cplx", [(64, 4, 0, False), (150, 8, 0, False), (200, 16, 0, False), (130, 32, 0, False),
                                        (97, 16, 2, False), (120, 8, 3, True), (90, 16, 0, True), (33, 32, 2, True),
                                        (5, 2, 0, False), (3, 1, 0, False)])
def test_rhess_invariants(n, r, p, cplx):
    print(f"[rhess] n={n} r={r} p={p} complex={cplx}", flush=True)
    A, B = inputs.dense_pencil(n, seed=n + r, complex_=cplx)
    Ao, Bo, Q, Z = _gpu_rhess(A, B, r, p)
    _check_invariants(A, B, Ao, Bo, Q, Z, r)
    e1 = np.zeros(n)
    e1[0] = 1.0
    assert np.array_equal(Z[:, 0], e1)
    assert fro(Q[:, 0] - B[:, 0] / Bo[0, 0]) <= 100 * n * EPS


@pytest.mark.parametrize("n,r,cplx", [(100, 8, False), (160, 16, False), (96, 32, False), (80, 8, True)])
def test_two_stage_matches_oracle_canonical(n, r, cplx):
    """The HT form of the full GPU path (ht_rhess then ht_stage2) equals the
    oracle's (rhess then stage2), in canonical form, to 1e-9."""
    from oracle import oracle as O
    print(f"[two-stage] n={n} r={r} complex={cplx}", flush=True)
    A, B = inputs.dense_pencil(n, seed=2 * n + r, complex_=cplx)
    H, T, Q, Z = _gpu_rhess(A, B, r, stage2=True)
    assert np.all(np.tril(H, -2) == 0) and np.all(np.tril(T, -1) == 0)
    A1, B1, Q1, Z1, _ = O.rhess(A, B, r, 8)
    Ho, To, Qo, Zo, _ = O.stage2(A1, B1, r, Q=Q1, Z=Z1)
    a = LR.canonical(H, T, Q, Z)
    b = LR.canonical(Ho, To, Qo, Zo)
    for x, y in zip(a, b):
        assert fro(x - y) / max(fro(y), 1.0) < 1e-9


def test_two_stage_saddle_point():
    """Singular B (saddle-point pencil, a quarter of infinite eigenvalues)
    through both GPU stages: invariants hold."""
    n, r = 96, 8
    A, B = inputs.saddle_point_pencil(n, 0.25, seed=4)
    H, T, Q, Z = _gpu_rhess(A, B, r, stage2=True)
    assert np.all(np.tril(H, -2) == 0) and np.all(np.tril(T, -1) == 0)
    bound = 100 * n * EPS
    assert fro(Q @ H @ Z.T - A) / fro(A) <= bound and fro(Q @ T @ Z.T - B) / fro(B) <= bound
    assert np.linalg.matrix_rank(T) == np.linalg.matrix_rank(B)


@pytest.mark.parametrize("n,r", [(1024, 16), (2048, 32)])
def test_rhess_invariants_large(n, r):
    ht = _ht()
    print(f"[rhess large] n={n} r={r}", flush=True)
    A, B = inputs.dense_pencil(n, seed=1)
    A0, B0 = ht.colmajor(A), ht.colmajor(B)
    Ad, Bd = A0.clone(), B0.clone()
    Qd = torch.eye(n, dtype=torch.float64, device="cuda").t().contiguous().t()
    Zd = Qd.clone()
    ht.rhess(Ad, Bd, r, Qd, Zd)
    torch.cuda.synchronize()
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    assert (torch.tril(Ad, -(r + 1)) == 0).all() and (torch.tril(Bd, -1) == 0).all()
    vals = [torch.linalg.norm(Qd.t() @ Qd - I).item(), torch.linalg.norm(Zd.t() @ Zd - I).item(),
            (torch.linalg.norm(Qd @ Ad @ Zd.t() - A0) / torch.linalg.norm(A0)).item(),
            (torch.linalg.norm(Qd @ Bd @ Zd.t() - B0) / torch.linalg.norm(B0)).item()]
    assert max(vals) <= 100 * n * EPS, vals


def _with_overlap(on, fn):
    ht = _ht()
    old = ht.set_knob(ht.KNOB_LOOKAHEAD, 2 if on else 0)      # 2: also below the automatic size limit
    try:
        return fn()
    finally:
        ht.set_knob(ht.KNOB_LOOKAHEAD, old)


@pytest.mark.parametrize("n,r,p,cplx,withq,withz", [
    (300, 4, 0, False, True, True), (500, 16, 0, False, True, True), (257, 8, 3, False, True, True),
    (700, 32, 2, False, True, True), (400, 16, 2, True, True, True), (333, 8, 0, True, True, True),
    (300, 16, 0, False, False, True), (300, 16, 0, False, True, False), (300, 16, 0, False, False, False),
    (1100, 16, 0, False, True, True), (40, 16, 0, False, True, True), (3, 1, 0, False, True, True)])
def test_rhess_overlap_is_bitwise_the_one_stream_order(n, r, p, cplx, withq, withz):
    """The three-stream schedule of stage one (Q and Z passes, and the rows of
    B that the next block factors do not read, on streams of their own) gives
    the same bits as the one-stream schedule.  The call runs on a side stream
    and the results are copied on that stream right after it, so a missing
    join of the other streams would show as a stale copy."""
    ht = _ht()
    print(f"[rhess overlap] n={n} r={r} p={p} complex={cplx} Q={withq} Z={withz}", flush=True)
    A, B = inputs.dense_pencil(n, seed=3 * n + r, complex_=cplx)

    def run():
        Ad, Bd = ht.colmajor(A), ht.colmajor(B)
        Qd = ht.colmajor(np.eye(n, dtype=A.dtype)) if withq else None
        Zd = ht.colmajor(np.eye(n, dtype=A.dtype)) if withz else None
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ht.rhess(Ad, Bd, r, Qd, Zd, p=p)
            outs = [x for x in (Ad, Bd, Qd, Zd) if x is not None]
            snap = [x.clone() for x in outs]
        torch.cuda.synchronize()
        for a, b in zip(outs, snap):
            assert torch.equal(a, b)
        return [ht.to_numpy(x) for x in outs]

    on = _with_overlap(True, run)
    off = _with_overlap(False, run)
    for a, b in zip(on, off):
        assert np.array_equal(a, b)
    if withq and withz:
        _check_invariants(A, B, on[0], on[1], on[2], on[3], r)


def test_rhess_invalid_arguments():
    ht = _ht()
    A = ht.colmajor(np.eye(64))
    with pytest.raises(ht.HTError) as e:
        ht.rhess(A, A.clone(), 16, p=5)          # 5 * 16 > 64
    assert e.value.code == -8
    with pytest.raises(ht.HTError) as e:
        ht.rhess(A, A.clone(), 40)
    assert e.value.code == 4
    assert ht.rhess_default_p(4096, 16) == 4 and ht.rhess_default_p(4096, 8) == 8 and ht.rhess_default_p(100, 32) == 2
