"""Pins for the oracle's PD-SDP / LR-PD-SDP iteration (Algorithms 1 and 2).

Values fixed by mathematics:
* max-cut on K_n: optimum n^2/4, dual y = -(n/4) 1 (Section 1.3 sign),
  optimal X = any PSD X with unit diagonal and X 1 = 0;
* max-cut on an odd cycle C_n: (n/2)(1 + cos(pi/n)); bipartite graphs: |E|;
* Goemans-Williamson sandwich: maxcut <= SDP <= maxcut / 0.87856;
* equipartition (Section 5.1): K_n gives n^2, C_n gives n(2 - 2cos(2 pi/n)),
  and 4 x (minimum bisection) bounds the relaxation from above;
* KKT at convergence (Section 2.1): dual feasibility, zero gap,
  complementarity; inequality duals <= 0 and zero on inactive rows.
"""
import math

import numpy as np
import pytest

import instances as I
import oracle as O


@pytest.mark.parametrize("n", [4, 7, 10])
def test_maxcut_complete_graph(n):
    prob = I.from_edges_maxcut(n, I.complete_edges(n))
    for full in (True, False):
        res = O.solve(prob, tol=1e-8, full_eig=full)
        assert res.status == O.CONVERGED
        assert -res.obj == pytest.approx(n * n / 4, rel=1e-6)
    # the dual is unique here: y = -(n/4) 1
    assert np.allclose(res.y, -n / 4, atol=1e-4)
    # optimal X are exactly the PSD X with unit diagonal and X 1 = 0
    assert np.allclose(np.diag(res.X), 1.0, atol=1e-5)
    assert np.allclose(res.X @ np.ones(n), 0.0, atol=1e-3)


@pytest.mark.parametrize("n", [5, 7, 9])
def test_maxcut_odd_cycle(n):
    prob = I.from_edges_maxcut(n, I.cycle_edges(n))
    res = O.solve(prob, tol=1e-8)
    assert res.status == O.CONVERGED
    assert -res.obj == pytest.approx(n / 2 * (1 + math.cos(math.pi / n)), rel=1e-6)
    ev = np.linalg.eigvalsh(res.X)
    assert np.sum(ev > 1e-4 * ev[-1]) == 2          # rank-2 optimum


def test_maxcut_bipartite():
    # complete bipartite K_{3,4} plus a path: bipartite, so SDP value = |E|
    left, right = range(3), range(3, 7)
    edges = np.array([(i, j) for i in left for j in right] + [(6, 7), (7, 8)])
    prob = I.from_edges_maxcut(9, edges)
    res = O.solve(prob, tol=1e-8)
    assert -res.obj == pytest.approx(len(edges), rel=1e-6)
    ev = np.linalg.eigvalsh(res.X)
    assert np.sum(ev > 1e-4 * ev[-1]) == 1          # rank-1 optimum


@pytest.mark.parametrize("seed", range(4))
def test_maxcut_goemans_williamson_sandwich(seed):
    n = 12
    edges = I.erdos_renyi_edges(n, 0.4, seed)
    prob = I.from_edges_maxcut(n, edges)
    res = O.solve(prob, tol=1e-7)
    mc = O.brute_force_maxcut(n, edges)
    sdp = -res.obj
    assert mc - 1e-4 <= sdp <= mc / 0.87856 + 1e-4


@pytest.mark.parametrize("seed", range(3))
def test_maxcut_kkt_at_convergence(seed):
    prob = I.maxcut(40, 0.15, seed)
    res = O.solve(prob, tol=1e-7)
    assert res.status == O.CONVERGED
    cert = O.certificate(prob, res.X, res.y)
    assert cert.rel_gap < 1e-5
    assert cert.dual_infeas < 1e-5
    assert cert.primal_infeas < 1e-6
    assert cert.lambda_min_X > -1e-8
    C = O.dense_sym_from_coo(prob.n, prob.c_i, prob.c_j, prob.c_v)
    S = C - np.diag(res.y)
    assert abs(np.sum(res.X * S)) < 1e-4 * (1 + abs(res.obj))   # complementarity
    lo, hi = O.maxcut_bracket(prob, res.X, res.y)
    assert lo <= res.obj + 1e-6 and lo - 1e-4 * abs(lo) <= hi


def test_lr_and_full_agree():
    prob = I.maxcut(50, 0.1, 0)
    a = O.solve(prob, tol=1e-7, full_eig=True)
    b = O.solve(prob, tol=1e-7, r0=1)
    assert a.obj == pytest.approx(b.obj, rel=1e-6)
    assert b.r < prob.n                              # the low-rank path stayed low-rank


@pytest.mark.parametrize("n", [6, 8])
def test_equipartition_complete_graph(n):
    prob = I.from_edges_equipartition(n, I.complete_edges(n))
    res = O.solve(prob, tol=1e-7)
    assert res.obj == pytest.approx(n * n, rel=1e-5)


@pytest.mark.parametrize("n", [8, 10, 12])
def test_equipartition_cycle(n):
    prob = I.from_edges_equipartition(n, I.cycle_edges(n))
    res = O.solve(prob, tol=1e-8)
    assert res.obj == pytest.approx(n * (2 - 2 * math.cos(2 * math.pi / n)), rel=1e-5)


@pytest.mark.parametrize("seed", range(3))
def test_equipartition_bisection_bound(seed):
    n = 10
    edges = I.erdos_renyi_edges(n, 0.4, seed)
    prob = I.from_edges_equipartition(n, edges)
    res = O.solve(prob, tol=1e-7)
    # <L, x x^T> = 4 * cut(x) for x in {-1,1}^n; the relaxation is a lower bound
    assert res.obj <= 4 * O.brute_force_min_bisection(n, edges) + 1e-4
    assert res.obj >= -1e-6


def test_inequality_rows_sign_and_activity():
    # minimize -X00 - X11  s.t.  X00 <= 1 (active), X11 <= 2 (active),
    # X00 + X11 <= 10 (inactive), X PSD.  Optimum -3, duals (-1, -1, 0).
    prob = I.Problem(n=2, m=0, p=3, c_i=[0, 1], c_j=[0, 1], c_v=[-1.0, -1.0],
                     a_row=[0, 1, 2, 2], a_i=[0, 1, 0, 1], a_j=[0, 1, 0, 1],
                     a_v=[1.0, 1.0, 1.0, 1.0], b=[], h=[1.0, 2.0, 10.0])
    res = O.solve(prob, tol=1e-9, full_eig=True)
    assert res.obj == pytest.approx(-3.0, abs=1e-6)
    assert np.allclose(res.y, [-1.0, -1.0, 0.0], atol=1e-5)
    assert res.dual_obj == pytest.approx(-3.0, abs=1e-6)


def test_two_by_two_closed_form():
    # minimize 2 X01 s.t. X00 = X11 = 1  ->  X = [[1,-1],[-1,1]], optimum -2
    prob = I.Problem(n=2, m=2, p=0, c_i=[0], c_j=[1], c_v=[1.0],
                     a_row=[0, 1], a_i=[0, 1], a_j=[0, 1], a_v=[1.0, 1.0],
                     b=[1.0, 1.0], h=[])
    res = O.solve(prob, tol=1e-9)
    assert res.obj == pytest.approx(-2.0, abs=1e-6)
    assert np.allclose(res.X, [[1, -1], [-1, 1]], atol=1e-5)


@pytest.mark.parametrize("kind,n", [("maxcut", 5), ("maxcut", 8), ("equip", 6)])
def test_warm_start_at_the_optimum_is_a_fixed_point(kind, n):
    # K_n: X* = n/(n-1) (I - 11^T/n) is optimal for both relaxations.  Max-cut:
    # y* = -(n/4) 1, S* = C - M*(y*) = 11^T/4.  Equipartition (rank-one row
    # <11^T, X> = 0): y* = (n 1, -1), S* = 0.  X* S* = 0, so one step of
    # Algorithm 1 from (X*, y*) returns (X*, y*) and the solve started there
    # stops at its first check.  y0 enters in the scaled rows (R2); the
    # all-ones row has Frobenius norm n, so a scaling slip breaks the fixed
    # point (an unscaled y0 runs 50 iterations and moves y by 0.14).
    # (Pins the oracle's start from a given point, the reference of the
    # library's warm start.)
    if kind == "maxcut":
        prob = I.from_edges_maxcut(n, I.complete_edges(n))
        ys = -n / 4 * np.ones(n)
        opt = -n * n / 4
    else:
        prob = I.from_edges_equipartition(n, I.complete_edges(n))
        ys = np.concatenate([n * np.ones(n), [-1.0]])
        opt = float(n * n)
    Xs = n / (n - 1) * (np.eye(n) - np.ones((n, n)) / n)
    ops = O.Operators(prob)
    res = O.solve(prob, tol=1e-8, full_eig=True, X0=Xs, y0=ys * ops.scale, ops=ops)
    assert res.iters == 10
    assert np.abs(res.X - Xs).max() <= 1e-12
    assert np.abs(res.y - ys).max() <= 1e-12 * max(1.0, np.abs(ys).max())
    assert res.obj == pytest.approx(opt, rel=1e-13)


def test_certificate_vanishes_at_known_optimum_only():
    n = 6
    prob = I.from_edges_maxcut(n, I.complete_edges(n))
    Xs = n / (n - 1) * (np.eye(n) - np.ones((n, n)) / n)
    ys = -n / 4 * np.ones(n)
    c = O.certificate(prob, Xs, ys)
    assert max(c.rho_p, c.rho_d, c.rel_gap, c.dual_infeas, c.primal_infeas) < 1e-12
    c2 = O.certificate(prob, Xs + 0.01 * np.eye(n), ys)
    assert max(c2.rho_p, c2.rho_d) > 1e-4
    c3 = O.certificate(prob, Xs, ys + 0.05)
    assert c3.dual_infeas > 1e-4 and max(c3.rho_p, c3.rho_d) > 1e-4


def test_snl_truth_is_feasible_without_noise():
    prob, pos, anchors = I.snl(30, seed=3, radius=0.6, noise=0.0, return_truth=True)
    Z = np.zeros((32, 32))
    Z[:2, :2] = np.eye(2)
    Z[:2, 2:] = pos.T
    Z[2:, :2] = pos
    Z[2:, 2:] = pos @ pos.T
    ops = O.Operators(prob, row_scaling=False)
    MZ = ops.apply(Z)
    assert np.allclose(MZ[:3], prob.b, atol=1e-12)
    g = MZ[3:]
    assert np.all(g <= prob.h + 1e-12)
    # noise-free rows: the two-sided band is +-10% around the true squared distance
    assert np.allclose(g[0::2], prob.h[0::2] / 1.1, rtol=1e-12)


def test_snl_small_recovers_positions():
    prob, pos, anchors = I.snl(12, seed=1, radius=0.9, noise=0.0, band=0.0, return_truth=True)
    res = O.solve(prob, tol=1e-7, max_iters=60000)
    assert res.status == O.CONVERGED
    Xhat = res.X[:2, 2:].T
    assert np.max(np.abs(Xhat - pos)) < 5e-3


def test_rank_path_doubles():
    prob = I.maxcut(50, 0.1, 0)
    res = O.solve(prob, tol=1e-4, r0=1)
    ranks = [r for _, r in res.rank_path]
    assert ranks[0] == 1
    assert all(b == min(2 * a, prob.n) for a, b in zip(ranks, ranks[1:]))
