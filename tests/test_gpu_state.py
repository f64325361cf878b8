"""Warm start through proxsdp_get_state / proxsdp_set_state on the GPU.

* Resumed iterates: K1 GPU iterations, the state (V, lambda, y) taken out,
  a fresh handle started from it and run K2 more iterations with converged
  eigensolves; the oracle runs the same K2 exact steps (Algorithm 1 with the
  rank-r projection) from X0 = V diag(lambda) V^T, y0 = y.  Bar as the other
  iterate tests: max |X_gpu - X_oracle| <= 1e-7 max(1, max |X|), same for y.
* Restart from a converged state: the resumed solve stops within its first
  residual window (50 iterations) with the objective of the first solve to
  the solve tolerance's objective band (1e-5 relative, as the solve parity
  tests).
* Invalid states are refused with PROXSDP_ERR_INVALID.
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


def _instance(kind, n, seed=7):
    if kind == "maxcut":
        return I.maxcut(n, 0.1, seed)
    if kind == "equip":
        return I.equipartition(n, 0.1, seed)
    return I.snl(n - 2, seed=seed, noise=0.0)


@pytest.mark.parametrize("kind,n,r,K1,K2", [("maxcut", 60, 4, 15, 15), ("equip", 50, 3, 15, 15),
                                            ("maxcut", 200, 4, 12, 12), ("snl", 102, 4, 20, 15)])
def test_resumed_iterates_match_oracle(torch_cuda, kind, n, r, K1, K2):
    from paper_1810_05231_amd import Solver
    _say("resume", kind, n, r, K1, K2)
    prob = _instance(kind, n)
    ops = O.Operators(prob)
    alpha = 0.95 / ops.norm()
    opts = dict(r0=r, alpha=alpha, check_every=5, window=1000, eig_strict=1, eig_tol=1e-13,
                max_iters=K1 + K2)
    a = Solver(prob, **opts)
    a.step(K1)
    V, lam, y = a.get_state()
    a.close()
    assert V.shape == (prob.n, lam.size) and lam.size <= r and np.all(lam >= 0)
    b = Solver(prob, **opts)
    b.set_state(V, lam, y)
    V2, lam2, y2 = b.get_state()
    assert np.array_equal(V2, V) and np.array_equal(lam2, lam)
    assert np.allclose(y2, y, rtol=1e-14, atol=0)
    info = b.step(K2)
    Xg, yg = b.solution(on_device=False)
    b.close()
    X = (V * lam) @ V.T
    ys = y * ops.scale
    C = ops.C()
    for _ in range(K2):
        out = O.pdhg_step(ops, C, X, ys, r, alpha)
        X, ys = out.X, out.y
    yo = ys / ops.scale
    scale = max(1.0, np.abs(X).max())
    _say("  dX", np.abs(Xg - X).max() / scale, "dy", np.abs(yg - yo).max())
    assert info["iters"] == K2
    assert np.abs(Xg - X).max() <= 1e-7 * scale
    assert np.abs(yg - yo).max() <= 1e-7 * max(1.0, np.abs(yo).max())
    assert info["eps_p"] == pytest.approx(out.eps_p, rel=1e-5, abs=1e-9)
    assert info["eps_d"] == pytest.approx(out.eps_d, rel=1e-5, abs=1e-9)


@pytest.mark.parametrize("kind,n,prec", [("maxcut", 150, 0), ("equip", 120, 1)])
def test_restart_from_converged_state(torch_cuda, kind, n, prec):
    from paper_1810_05231_amd import Solver
    prob = I.maxcut(n, 0.05, 3) if kind == "maxcut" else I.equipartition(n, 0.05, 3)
    a = Solver(prob, precision=prec)
    ia = a.solve()
    V, lam, y = a.get_state()
    a.close()
    b = Solver(prob, precision=prec)
    b.set_state(V, lam, y)
    ib = b.solve()
    _say("  first", ia["iters"], repr(ia["obj"]), " resumed", ib["iters"], repr(ib["obj"]), ib["r"])
    assert ia["status_name"] == ib["status_name"] == "converged"
    assert ib["iters"] <= 50
    assert ib["obj"] == pytest.approx(ia["obj"], rel=1e-5)
    b.close()


def test_invalid_states_are_refused(torch_cuda):
    from paper_1810_05231_amd import Solver
    from paper_1810_05231_amd._lib import ProxSDPError
    prob = I.snl(40, seed=2, noise=0.0)
    s = Solver(prob, r0=2)
    n, rows, m = prob.n, prob.m + prob.p, prob.m
    V = np.ones((n, 2))
    with pytest.raises(ProxSDPError):
        s.set_state(V, np.array([1.0, -1.0]))          # X0 not PSD
    with pytest.raises(ProxSDPError):
        s.set_state(np.full((n, 2), np.nan), np.array([1.0, 1.0]))
    y = np.zeros(rows)
    y[m] = 1.0                                          # positive inequality dual
    with pytest.raises(ProxSDPError):
        s.set_state(V, np.array([1.0, 1.0]), y)
    with pytest.raises(ProxSDPError):
        s.set_state(np.ones((n, 65)), np.ones(65))      # beyond the factor storage
    # the handle still works after the refusals, and r = 0 is X0 = 0
    s.set_state(np.zeros((n, 0)), np.zeros(0), None)
    info = s.step(10)
    assert info["iters"] == 10
    s.close()
