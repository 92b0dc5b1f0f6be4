"""GPU tests of the request loop (continuous batching of complex128
reductions, HBM-footprint admission): every request completes with a valid
Hessenberg-triangular decomposition, requests overlap on the device, the
accounted footprint stays within the budget, and a request's result is the
same alone and in the mix (to 1e-9 relative: small requests run in the
batched launch in the mix and alone through the single-pencil path)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _check(req, res):
    import paper_2301_07964_amd.serving as S
    H, T, Q, Z = res
    A, B, _, _ = S._synthesize(req, torch.device("cuda:0"))
    if req.dense:
        # a dense request ends in HT form of the dense pencil
        pass
    n = req.n
    I = torch.eye(n, dtype=torch.complex128, device="cuda")
    assert (torch.tril(H, -2) == 0).all() and (torch.tril(T, -1) == 0).all()
    vals = [torch.linalg.norm(Q.conj().t() @ Q - I).item(), torch.linalg.norm(Z.conj().t() @ Z - I).item(),
            (torch.linalg.norm(Q @ H @ Z.conj().t() - A) / torch.linalg.norm(A)).item(),
            (torch.linalg.norm(Q @ T @ Z.conj().t() - B) / torch.linalg.norm(B)).item()]
    assert max(vals) <= 100 * n * EPS, (req, vals)


def test_continuous_batching_results_and_overlap():
    import paper_2301_07964_amd.serving as S
    trace = S.make_trace(20, rate=200.0, seed=3, nhi=768)
    print(f"[serving] n={[q.n for q in trace]} dense={[int(q.dense) for q in trace]}", flush=True)
    eng = S.Engine("continuous", slots=4, small_n=256, keep_results=True)
    eng.run(trace, time_limit=240)
    assert all(np.isfinite(q.done) and q.done >= q.arrival for q in trace)
    assert eng.max_inflight > 1
    assert eng.peak_bytes <= eng.budget
    for q in trace:
        _check(q, q.result)
    # alone vs in the mix: every request of the trace
    for q in trace:
        alone = S.Request(q.rid, 0.0, q.n, q.r, q.dense, q.seed)
        S.Engine("fifo", keep_results=True).run([alone], time_limit=120)
        for x, y in zip(q.result, alone.result):
            d = (torch.linalg.norm(x - y) / max(torch.linalg.norm(y).item(), 1.0)).item()
            assert d <= 1e-9, (q, d)


def test_admission_respects_a_small_budget():
    import paper_2301_07964_amd.serving as S
    trace = S.make_trace(8, rate=1000.0, seed=4, nhi=512)
    need = max(S.footprint(q) for q in trace)
    eng = S.Engine("continuous", slots=4, small_n=0, budget_bytes=int(1.5 * need))
    eng.run(trace, time_limit=120)
    assert eng.peak_bytes <= eng.budget
    assert all(np.isfinite(q.done) for q in trace)


def test_fifo_serves_in_arrival_order():
    import paper_2301_07964_amd.serving as S
    trace = S.make_trace(6, rate=1000.0, seed=5, nhi=384)
    S.Engine("fifo").run(trace, time_limit=120)
    adm = [q.admitted for q in sorted(trace, key=lambda q: q.arrival)]
    assert adm == sorted(adm)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _oracle_result(req, A, B, perturb=False):
    """The oracle's reduction of a served request's pencil: stage two for an
    r-HT request; stage one (QR of B, blocked reduction, p = 8) then stage two
    for a dense one.  perturb: the band of H (or A) scaled by 1 + 1e-15 N(0,1)
    entry-wise first (the sensitivity floor)."""
    from oracle import oracle as O
    if perturb:
        rng = np.random.default_rng(1)
        P = rng.standard_normal(A.shape) + 1j * rng.standard_normal(A.shape)
        A = A + 1e-15 * np.abs(A) * P
    if req.dense:
        A1, B1, Q1, Z1, _ = O.rhess(A, B, req.r, 8)
        return O.stage2(A1, B1, req.r, Q=Q1, Z=Z1)[:4]
    return O.stage2(A, B, req.r)[:4]


def test_served_results_match_oracle():
    """A parity sample of 32 served requests (continuous batching, complex128,
    n log-uniform on [64, 640] with its largest n included, 20% dense): every
    served H, T, Q, Z against the oracle's reduction of the same pencil.  r-HT
    requests are compared entry by entry; dense requests in canonical form (the
    HT form with Q e1 fixed is unique up to a unimodular diagonal scaling,
    while stage one's intermediate r-HT form depends on its blocking).  Bound:
    1e-9, or 10x the oracle's own response to a 1e-15 relative perturbation of
    the input where that is larger (complex pencils of the generator are
    sensitive)."""
    import paper_2301_07964_amd.serving as S
    from oracle import oracle as O
    from tests import lapack_ref as LR
    O.set_threads(max(1, min(16, O.host_cores())))
    trace = S.make_trace(32, rate=100.0, seed=7, nhi=640)
    print(f"[serving parity] n={[q.n for q in trace]} dense={[int(q.dense) for q in trace]}", flush=True)
    eng = S.Engine("continuous", slots=4, small_n=256, keep_results=True)
    eng.run(trace, time_limit=240)
    worst = []
    for q in trace:
        A, B, _, _ = [x.cpu().numpy() for x in S._synthesize(q, torch.device("cuda:0"))]
        got = [x.cpu().numpy() for x in q.result]
        ref = _oracle_result(q, A, B)
        ref2 = _oracle_result(q, A, B, perturb=True)
        if q.dense:
            got, ref, ref2 = LR.canonical(*got), LR.canonical(*ref), LR.canonical(*ref2)
        floor = max(_rel(a, b) for a, b in zip(ref2, ref))
        err = max(_rel(a, b) for a, b in zip(got, ref))
        worst.append((err, floor, q.n, q.r, q.dense))
        assert err <= max(1e-9, 10 * floor), (q, err, floor)
    print("[serving parity] worst (err, floor, n, r, dense):", sorted(worst)[-3:], flush=True)
    assert max(q.n for q in trace) == max(w[2] for w in worst)
