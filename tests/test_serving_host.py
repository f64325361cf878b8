"""Host-side pieces of the serving form (no GPU): the workload generator, the
latency percentile and the request loop's admission bookkeeping."""
import numpy as np

import instances as I
from paper_1810_05231_amd.serving import percentile


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert percentile(xs, 50) == 50
    assert percentile(xs, 99) == 99
    assert percentile(xs, 100) == 100
    assert percentile([3.0], 99) == 3.0
    assert percentile([5, 1, 4, 2, 3], 50) == 3


def test_serving_stream_shape_and_seed():
    a = I.serving_stream(40, seed=1, rate=10.0)
    b = I.serving_stream(40, seed=1, rate=10.0)
    assert [(r[0], r[1], r[2].n, r[2].name) for r in a] == [(r[0], r[1], r[2].n, r[2].name) for r in b]
    ns = np.array([r[2].n for r in a])
    assert ns.min() >= 100 and ns.max() <= 2000
    arr = np.array([r[1] for r in a])
    assert np.all(np.diff(arr) >= 0) and arr[0] > 0
    kinds = {r[2].name.split("_")[0] for r in a}
    assert kinds == {"maxcut", "equip"}
    # G(n, 8/n): mean degree about 8
    deg = np.mean([2 * r[2].meta["edges"] / r[2].n for r in a])
    assert 6.5 < deg < 9.5


def test_serving_stream_poisson_rate():
    a = I.serving_stream(400, seed=2, rate=20.0, n_lo=100, n_hi=120)
    arr = np.array([r[1] for r in a])
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 1 / 20.0) < 0.2 / 20.0
    z = I.serving_stream(5, seed=2, rate=None, n_lo=100, n_hi=120)
    assert all(r[1] == 0.0 for r in z)


# ------------------------------------------------------------- request loop
# The loop's bookkeeping (arrival order, footprint budget, slots, completion)
# with the device calls replaced by a stand-in whose solves need a fixed
# number of iterations each; the footprints are the library's own
# (proxsdp_workspace_size is host-only).
class _FakeSolver:
    created = []

    def __init__(self, prob, device=None, stream=None, **opts):
        self.n = prob.n
        self.need = 40 + prob.n // 5
        self.iters = 0
        self.closed = False
        _FakeSolver.created.append(prob.name)

    def close(self):
        self.closed = True


def _fake_step_many(solvers, n_iters, until_any_stops=False):
    adv = n_iters
    if until_any_stops:
        adv = min(n_iters, min(s.need - s.iters for s in solvers))
    out = []
    for s in solvers:
        s.iters += min(adv, s.need - s.iters)
        done = s.iters == s.need
        out.append(dict(status_name="converged" if done else "running", iters=s.iters,
                        obj=float(s.n), rho_p=0.0, rho_d=0.0))
    return out


def _server(monkeypatch, **kw):
    import torch
    import paper_1810_05231_amd.serving as S

    class _Stream:
        def __init__(self, device=None):
            pass

    monkeypatch.setattr(torch.cuda, "Stream", _Stream)
    monkeypatch.setattr(S, "Solver", _FakeSolver)
    monkeypatch.setattr(S, "step_many", _fake_step_many)
    _FakeSolver.created = []
    return S.Server(device="cpu", **kw)


def _clock():
    t = [0.0]

    def clock():
        t[0] += 0.001
        return t[0]
    return clock


def test_server_admits_in_arrival_order_within_budget_and_slots(monkeypatch):
    from paper_1810_05231_amd.serving import Request
    reqs = I.serving_stream(9, seed=4, rate=None, n_lo=100, n_hi=300)
    srv = _server(monkeypatch, max_slots=3, round_iters=25)
    fps = [srv.footprint(p) for _, _, p in reqs]
    srv.budget = sorted(fps)[-1] + sorted(fps)[-2]      # room for about two at a time
    results = srv.run([Request(rid, 0.0, p) for rid, _, p in reqs], clock=_clock())
    assert sorted(r.rid for r in results) == [rid for rid, _, _ in reqs]
    assert all(r.status == "converged" for r in results)
    # each solve needed its own number of iterations, whatever ran beside it
    for r in results:
        assert r.iters == 40 + r.n // 5
    assert srv.peak_bytes <= srv.budget and srv.peak_slots <= 3
    assert srv.peak_slots >= 2
    # admission follows arrival order (ties by request id)
    assert _FakeSolver.created == [p.name for _, _, p in reqs]
    # later requests waited for memory or a slot
    assert max(r.admitted for r in results) > min(r.admitted for r in results)


def test_server_rejects_a_request_above_the_budget(monkeypatch):
    from paper_1810_05231_amd.serving import Request
    reqs = I.serving_stream(2, seed=5, rate=None, n_lo=150, n_hi=160)
    srv = _server(monkeypatch, max_slots=2)
    srv.budget = min(srv.footprint(p) for _, _, p in reqs) - 1
    import pytest
    with pytest.raises(ValueError):
        srv.run([Request(rid, 0.0, p) for rid, _, p in reqs], clock=_clock())
