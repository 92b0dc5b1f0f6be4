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
    # alone vs in the mix
    for q in [t for t in trace if not t.dense][:3] + [t for t in trace if t.dense][:2]:
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
