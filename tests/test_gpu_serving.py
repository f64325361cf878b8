"""Serving form on the GPU: continuous batching through proxsdp_step_many.

Each solve runs on its own stream with its whole state resident in its own
workspace, and every reduction in the library has a fixed order, so a solve
must give the same iterates alone and in the mix: the test requires the same
status and iteration count and objectives equal to 1e-12 relative.  The
precision form (FP32 storage of W) is the serving configuration.
"""
import sys

import numpy as np
import pytest

import instances as I
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests():
    # small sizes so that the test is quick; mixed kinds and sizes
    reqs = I.serving_stream(6, seed=3, n_lo=100, n_hi=400, mean_degree=8.0, rate=None)
    return reqs


@pytest.mark.parametrize("kind,n,prec", [("maxcut", 300, 0), ("equip", 200, 1), ("maxcut", 400, 2)])
def test_graph_rounds_match_eager(torch_cuda, kind, n, prec):
    """Rounds replayed from captured HIP graphs (many replays, with the control
    checks' synchronisations and host reads between them) give bitwise the
    eager launches' results."""
    from paper_1810_05231_amd.solver import Solver
    prob = I.maxcut(n, 0.05, 11) if kind == "maxcut" else I.equipartition(n, 0.05, 11)
    a = Solver(prob, precision=prec)
    ia = a.solve()
    b = Solver(prob, precision=prec, graphs=1, stream=torch_cuda.cuda.Stream())
    ib = b.solve()
    _say("  eager", ia["iters"], repr(ia["obj"]), " graphs", ib["iters"], repr(ib["obj"]))
    assert ia["status_name"] == ib["status_name"] == "converged"
    assert ia["iters"] == ib["iters"] and ia["passes"] == ib["passes"]
    assert ib["obj"] == ia["obj"]
    Xa, ya = a.solution(on_device=False)
    Xb, yb = b.solution(on_device=False)
    assert np.array_equal(Xa, Xb) and np.array_equal(ya, yb)
    a.close()
    b.close()


def test_step_many_matches_step(torch_cuda):
    """proxsdp_step_many over several handles == proxsdp_step on each."""
    from paper_1810_05231_amd.solver import Solver, step_many
    reqs = _requests()[:3]
    streams = [torch_cuda.cuda.Stream() for _ in reqs]
    alone = []
    for _, _, prob in reqs:
        s = Solver(prob, precision=1)
        info = s.step(200)
        alone.append(info)
        s.close()
    mix = [Solver(prob, stream=st, precision=1, graphs=1) for (_, _, prob), st in zip(reqs, streams)]
    infos = step_many(mix, 200)
    for a, b in zip(alone, infos):
        _say("  alone", a["iters"], repr(a["obj"]), " mix", b["iters"], repr(b["obj"]))
        assert a["iters"] == b["iters"]
        assert b["obj"] == pytest.approx(a["obj"], rel=1e-12, abs=1e-12)
    for s in mix:
        s.close()


def test_serving_alone_vs_mix(torch_cuda):
    from paper_1810_05231_amd.serving import Request, Server
    from paper_1810_05231_amd.solver import Solver
    reqs = _requests()
    alone = {}
    for rid, _, prob in reqs:
        s = Solver(prob, precision=1)
        info = s.solve()
        alone[rid] = info
        s.close()
    # budget for about three of the six at a time: later requests queue for memory
    srv = Server(max_slots=4, precision=1, graphs=1)
    fps = sorted(srv.footprint(p) for _, _, p in reqs)
    srv.budget = fps[-1] + fps[-2] + fps[-3]
    certs = {}

    def on_done(res, solver):
        X, y = solver.solution(on_device=False)
        prob = [p for rid, _, p in reqs if rid == res.rid][0]
        certs[res.rid] = O.certificate(prob, X, y)

    results = srv.run([Request(rid, 0.0, prob) for rid, _, prob in reqs], on_done=on_done)
    assert len(results) == len(reqs)
    assert srv.peak_bytes <= srv.budget
    _say("  peak slots", srv.peak_slots, "peak bytes", srv.peak_bytes, "budget", srv.budget)
    for res in results:
        a = alone[res.rid]
        c = certs[res.rid]
        _say("  rid", res.rid, "n", res.n, res.status, res.iters, repr(res.obj), "alone",
             a["iters"], repr(a["obj"]), "cert", c.rho_p, c.rho_d)
        assert res.status == "converged" and a["status_name"] == "converged"
        assert res.iters == a["iters"]
        assert res.obj == pytest.approx(a["obj"], rel=1e-12, abs=1e-12)
        assert max(c.rho_p, c.rho_d) <= 2e-4
    # requests beyond the budget had to wait for a finished solve
    assert max(r.admitted for r in results) > 0.0
