"""The continuous-batching server on the GPU: each result equals the same
product computed alone, within rounding, whatever it was batched with; the
memory budget admits requests one slot at a time instead of failing."""
import threading

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _geoms(mf):
    out = []
    for v, t in (synth.icosphere(6, 0.5), synth.ellipsoid(10, (0.9, 0.7, 0.5)),
                 synth.rounded_box((1.0, 1.0, 0.5), 0.1, 0.08)):
        out.append(mf.Geometry(v, t, max_rhs=16).precompute())
    return out


@pytest.mark.parametrize("dtype,tol", [("complex128", 1e-12), ("complex64", 2e-5)])
def test_alone_equals_mixed(dtype, tol):
    torch = _torch()
    import paper_2210_04892_amd as mf
    geoms = _geoms(mf)
    rng = np.random.default_rng(21)
    tdt = getattr(torch, dtype)
    reqs = []
    for i in range(30):
        gi = int(rng.integers(len(geoms)))
        nr = int(rng.integers(1, 7))
        n2 = 2 * geoms[gi].n_rwg
        x = torch.from_numpy(rng.standard_normal((nr, n2)) + 1j * rng.standard_normal((nr, n2))).to(tdt).cuda()
        reqs.append((gi, x, "C" if i % 3 else "EM"))
    srv = mf.Server(streams=3, max_batch_rhs=16)
    ys = [torch.empty_like(x) for _, x, _ in reqs]
    tickets = [None] * len(reqs)

    def client(k):
        for i in range(k, len(reqs), 2):
            gi, x, op = reqs[i]
            tickets[i] = srv.submit(geoms[gi], x, ys[i], op=op)

    th = [threading.Thread(target=client, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    batches = [srv.wait(t)[1] for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["requests"] == len(reqs)
    assert max(batches) > 6 or st["launches"] < len(reqs)      # some requests shared a product
    for (gi, x, op), y in zip(reqs, ys):
        alone = geoms[gi].matvec(x.t(), op=op).t()
        d = float(torch.linalg.norm(alone - y) / torch.linalg.norm(alone))
        assert d <= tol, d


def test_budget_admission():
    torch = _torch()
    import paper_2210_04892_amd as mf
    geoms = _geoms(mf)
    x = torch.randn(4, 2 * geoms[0].n_rwg, dtype=torch.complex64, device="cuda")
    # room for one slot only: requests are served one product at a time
    probe = mf.Server(streams=1, max_batch_rhs=16)
    y = torch.empty_like(x)
    probe.wait(probe.submit(geoms[0], x, y))
    one = probe.stats()["arena_bytes"]
    probe.close()
    srv = mf.Server(streams=4, max_batch_rhs=16, hbm_budget_bytes=int(one * 1.5))
    ys = [torch.empty_like(x) for _ in range(8)]
    ts = [srv.submit(geoms[0], x, ys[i]) for i in range(8)]
    for t in ts:
        srv.wait(t)
    assert srv.stats()["arena_bytes"] <= int(one * 1.5)
    ref = geoms[0].matvec(x.t()).t()
    for y in ys:
        assert float(torch.linalg.norm(y - ref) / torch.linalg.norm(ref)) < 2e-5
    srv.close()
    # a budget below one slot can never admit the request
    srv = mf.Server(streams=2, max_batch_rhs=16, hbm_budget_bytes=1024)
    with pytest.raises(mf.MlfmaError) as e:
        srv.wait(srv.submit(geoms[0], x, torch.empty_like(x)))
    assert e.value.code == -3
    srv.close()


def test_submit_is_ordered_after_the_callers_stream():
    """x is produced on torch's current stream by work still queued when the
    request is submitted (a long chain of products followed by the copy that
    writes x): the server must read x only after that work, so the served
    result equals the product of the final x computed alone."""
    torch = _torch()
    import paper_2210_04892_amd as mf
    geoms = _geoms(mf)
    g = geoms[1]
    n2 = 2 * g.n_rwg
    x_true = torch.from_numpy(synth.gaussian_coeffs(n2, 3, 61).T.copy()).to(torch.complex64).cuda()
    srv = mf.Server(streams=2, max_batch_rhs=16)
    for rep in range(3):
        x = torch.zeros_like(x_true)
        y = torch.empty_like(x_true)
        torch.cuda.synchronize()
        a = torch.randn(2048, 2048, device="cuda")
        for _ in range(40):                  # about 20 ms of queued work ahead of the copy
            a = torch.tanh(a @ a) * 0.5
        x.copy_(x_true + 0 * a[0, 0])        # written only after the chain
        t = srv.submit(g, x, y)
        srv.wait(t)
        alone = g.matvec(x_true.t()).t()
        torch.cuda.synchronize()
        d = float(torch.linalg.norm(alone - y) / torch.linalg.norm(alone))
        print("[gpu] submit after queued work, rep %d: rel diff %.2e" % (rep, d), flush=True)
        assert d <= 2e-5, d
    srv.close()


def test_destroy_with_pending_requests():
    """Requests still queued when the server is destroyed fail cleanly and
    a thread blocked waiting for one of them returns (no use after free)."""
    torch = _torch()
    import paper_2210_04892_amd as mf
    geoms = _geoms(mf)
    g = geoms[2]
    x = torch.randn(2, 2 * g.n_rwg, dtype=torch.complex64, device="cuda")
    srv = mf.Server(streams=1, max_batch_rhs=2)
    ys = [torch.empty_like(x) for _ in range(12)]
    tickets = [srv.submit(g, x, y) for y in ys]
    outcome = {}

    def waiter():
        try:
            srv.wait(tickets[-1])
            outcome["rc"] = 0
        except mf.MlfmaError as e:
            outcome["rc"] = e.code

    th = threading.Thread(target=waiter)
    th.start()
    srv.close()
    th.join(timeout=60)
    assert not th.is_alive()
    assert outcome["rc"] in (0, -5)
    torch.cuda.synchronize()
