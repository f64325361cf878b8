"""Pins for the oracle's residuals (Section 2.2) and Algorithm 2's rank test.

Each value below is worked out by hand from the iteration on a 1 x 1 problem
(the PSD cone of S^1 is x >= 0, aproj is max(., 0), M is the identity), not
by calling the oracle's own formulas:

  equality row   min -x  s.t. x = 1      (C = -1, b = 1, ||M|| = 1, alpha = 0.95)
    step 1 from (0, 0):  W = alpha = 0.95, x1 = 0.95,
                         y1 = alpha (1 - 2 x1) = -0.855,
                         eps_p = |x1/alpha + y1| = 0.145,
                         eps_d = |y1/alpha + x1| = 0.05
    step 2:              W = x1 - alpha (C - y1) = 1.08775 = x2,
                         y2 = y1 + alpha (1 - (2 x2 - x1)) = -1.069225,
                         eps_p = |0.13775/0.95 - 0.214225| = 0.069225,
                         eps_d = |-0.2255 + 0.13775| = 0.08775
  inequality row min -x  s.t. x <= 0.5   (h = 0.5)
    step 1 from (0, 0):  x1 = 0.95, u = alpha (0.5 - 1.9) = -1.33, y1 = min(0, u) = -1.33,
                         eps_p = |1 - 1.33| = 0.33, eps_d = |-1.4 + 0.95| = 0.45

A sign slip in either residual (the dual sign of Section 1.3 against
Algorithm 1's) changes these numbers (e.g. eps_p = 1.855 instead of 0.145).

Rank test (Algorithm 2, (n - r) lambda_r <= eps_lambda with lambda_r the r-th
largest eigenvalue of the projected matrix): the max-cut relaxation of an odd
cycle has a unique optimum of rank 2 (Section 5 pins in test_oracle_solve), so
at r = 2 the 2nd eigenvalue is positive and the test must fail; r doubles to
4, where lambda_4 <= 0.  The rank path therefore ends at 4.  Reading
lambda_{r+1} instead would stop at r = 2.
"""
import math

import numpy as np
import pytest

import instances as I
import oracle as O


def _one_by_one(eq: bool):
    if eq:
        return I.Problem(n=1, m=1, p=0, c_i=[0], c_j=[0], c_v=[-1.0], a_row=[0], a_i=[0],
                         a_j=[0], a_v=[1.0], b=[1.0], h=[])
    return I.Problem(n=1, m=0, p=1, c_i=[0], c_j=[0], c_v=[-1.0], a_row=[0], a_i=[0], a_j=[0],
                     a_v=[1.0], b=[], h=[0.5])


def test_residuals_one_step_equality_row():
    prob = _one_by_one(True)
    ops = O.Operators(prob)
    assert ops.norm() == 1.0
    out = O.pdhg_step(ops, ops.C(), np.zeros((1, 1)), np.zeros(1), 1, 0.95)
    assert out.X[0, 0] == pytest.approx(0.95, abs=1e-15)
    assert out.y[0] == pytest.approx(-0.855, abs=1e-15)
    assert out.eps_p == pytest.approx(0.145, abs=1e-14)
    assert out.eps_d == pytest.approx(0.05, abs=1e-14)
    out2 = O.pdhg_step(ops, ops.C(), out.X, out.y, 1, 0.95, out.MX)
    assert out2.X[0, 0] == pytest.approx(1.08775, abs=1e-14)
    assert out2.y[0] == pytest.approx(-1.069225, abs=1e-14)
    assert out2.eps_p == pytest.approx(0.069225, abs=1e-14)
    assert out2.eps_d == pytest.approx(0.08775, abs=1e-14)


def test_residuals_one_step_inequality_row():
    prob = _one_by_one(False)
    ops = O.Operators(prob)
    out = O.pdhg_step(ops, ops.C(), np.zeros((1, 1)), np.zeros(1), 1, 0.95)
    assert out.X[0, 0] == pytest.approx(0.95, abs=1e-15)
    assert out.y[0] == pytest.approx(-1.33, abs=1e-14)
    assert out.eps_p == pytest.approx(0.33, abs=1e-14)
    assert out.eps_d == pytest.approx(0.45, abs=1e-14)


def test_solve_reports_the_last_step_residuals():
    # two iterations with check_every = 2: the reported residuals and rho are
    # the second step's (rho_p = eps_p / (1 + ||C||_F), ||C||_F = 1;
    # rho_d = eps_d / (1 + ||b||), ||b|| = 1)
    prob = _one_by_one(True)
    res = O.solve(prob, tol=1e-12, check_every=2, window=2, max_iters=2, full_eig=True)
    assert res.iters == 2
    assert res.eps_p == pytest.approx(0.069225, abs=1e-14)
    assert res.eps_d == pytest.approx(0.08775, abs=1e-14)
    assert res.rho_p == pytest.approx(0.069225 / 2, abs=1e-14)
    assert res.rho_d == pytest.approx(0.08775 / 2, abs=1e-14)


@pytest.mark.parametrize("n", [5, 7])
def test_rank_test_reads_lambda_r(n):
    prob = I.from_edges_maxcut(n, I.cycle_edges(n))
    res = O.solve(prob, tol=1e-8, r0=1)
    assert res.status == O.CONVERGED
    ranks = [r for _, r in res.rank_path]
    assert ranks == [1, 2, 4]
    assert res.r == 4
    # the optimum itself has rank 2 (two eigenvalues above the noise)
    ev = np.linalg.eigvalsh(res.X)
    assert int(np.sum(ev > 1e-4 * ev[-1])) == 2
    # and the returned lambda_r of the projected matrix is non-positive
    assert res.lam_r <= 0.0


def test_rank_test_passes_at_sufficient_start():
    # started at r0 = 4 the first converged check passes the rank test: no update
    prob = I.from_edges_maxcut(7, I.cycle_edges(7))
    res = O.solve(prob, tol=1e-8, r0=4)
    assert res.status == O.CONVERGED
    assert [r for _, r in res.rank_path] == [4]


# -------------------------------------------- brute force and the bracket on K_n
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8])
def test_brute_force_maxcut_complete_graph(n):
    # K_n: the best cut puts floor(n/2) vertices on one side
    assert O.brute_force_maxcut(n, I.complete_edges(n)) == (n // 2) * ((n + 1) // 2)


@pytest.mark.parametrize("n", [4, 6, 8])
def test_brute_force_min_bisection_complete_and_cycle(n):
    # K_n: every bisection cuts (n/2)^2 edges; C_n: the best bisection cuts 2 edges
    assert O.brute_force_min_bisection(n, I.complete_edges(n)) == (n // 2) ** 2
    assert O.brute_force_min_bisection(n, I.cycle_edges(n)) == 2


@pytest.mark.parametrize("n", [4, 5, 8])
def test_maxcut_bracket_closed_forms_on_complete_graph(n):
    # C = -L/4 with L = n I - 1 1^T.  At y* = -(n/4) 1 the slack C - Diag(y*) = 1 1^T / 4
    # has lambda_min = 0, so lower = sum(y*) = -n^2/4.  X* = n/(n-1)(I - 1 1^T/n) has a
    # unit diagonal, so upper = <C, X*> = -n^2/4.
    prob = I.from_edges_maxcut(n, I.complete_edges(n))
    Xs = n / (n - 1) * (np.eye(n) - np.ones((n, n)) / n)
    ys = -n / 4 * np.ones(n)
    lo, hi = O.maxcut_bracket(prob, Xs, ys)
    assert lo == pytest.approx(-n * n / 4, abs=1e-12)
    assert hi == pytest.approx(-n * n / 4, abs=1e-12)
    # the upper side rescales to a unit diagonal: 2 X* gives the same value
    lo2, hi2 = O.maxcut_bracket(prob, 2.0 * Xs, ys)
    assert hi2 == pytest.approx(-n * n / 4, abs=1e-12)
    # the identity is feasible: <C, I> = -trace(L)/4 = -n (n - 1)/4
    _, hi3 = O.maxcut_bracket(prob, np.eye(n), ys)
    assert hi3 == pytest.approx(-n * (n - 1) / 4, abs=1e-12)
    # y = y* - d 1 is dual feasible (slack 1 1^T/4 + d I >= 0): lower = sum(y)
    d = 0.3
    lo4, _ = O.maxcut_bracket(prob, Xs, ys - d)
    assert lo4 == pytest.approx(-n * n / 4 - n * d, abs=1e-12)
    # y = y* + d e_1 is not: the slack has lambda_min = -d + O(d^2) < 0, which
    # enters as n * lambda_min (the shift of y that restores feasibility)
    e1 = np.zeros(n)
    e1[0] = d
    lo5, _ = O.maxcut_bracket(prob, Xs, ys + e1)
    C = -0.25 * (n * np.eye(n) - np.ones((n, n)))
    lmin = float(np.linalg.eigvalsh(C - np.diag(ys + e1))[0])
    assert lmin < 0
    assert lo5 == pytest.approx(-n * n / 4 + d + n * lmin, abs=1e-12)
    assert lo5 < -n * n / 4


@pytest.mark.parametrize("n", [5, 7])
def test_rank_test_lambda_r_plus_1_stops_at_the_rank(n):
    # the first excluded eigenvalue lambda_3 of the projected matrix is <= 0 at
    # the rank-2 optimum, so the lambda_{r+1} reading stops at r = 2
    prob = I.from_edges_maxcut(n, I.cycle_edges(n))
    res = O.solve(prob, tol=1e-8, rank_test="lambda_r_plus_1")
    assert res.status == O.CONVERGED
    assert [r for _, r in res.rank_path] == [1, 2]
    assert -res.obj == pytest.approx(n / 2 * (1 + math.cos(math.pi / n)), rel=1e-6)


@pytest.mark.parametrize("n", [5, 7])
def test_rank_cap_stops_with_rank_limit(n):
    # r_max = 2 < n: the residual converges at r = 2 but the lambda_r test fails
    # (lambda_2 > 0 at a rank-2 optimum) and r cannot double: RANK_LIMIT.  The
    # saved X_[r] are feasible (unit diagonal, PSD); X_[2] is in fact optimal
    # here, which the literal lambda_r test cannot see.
    prob = I.from_edges_maxcut(n, I.cycle_edges(n))
    res = O.solve(prob, tol=1e-8, r_max=2)
    assert res.status == O.RANK_LIMIT
    assert res.r == 2
    assert [s[1] for s in res.saved] == [1, 2]
    for _, r, Xr, yr in res.saved:
        assert np.allclose(np.diag(Xr), 1.0, atol=1e-6)
        assert np.linalg.eigvalsh(Xr)[0] >= -1e-10
        assert np.linalg.matrix_rank(Xr, tol=1e-6) <= r
    assert -res.obj == pytest.approx(n / 2 * (1 + math.cos(math.pi / n)), rel=1e-6)
    # X_[1] is a rank-one feasible point: +-1 vector outer product, so its cut
    # value is an integer cut, at most the maximum cut (n - 1 for odd cycles)
    X1 = res.saved[0][2]
    L = np.zeros((n, n))
    for a, b in I.cycle_edges(n):
        L[a, a] += 1
        L[b, b] += 1
        L[a, b] -= 1
        L[b, a] -= 1
    cut1 = float(np.sum(-0.25 * L * X1))
    assert -cut1 <= n - 1 + 1e-6


def test_rank_test_option_is_checked():
    prob = I.from_edges_maxcut(5, I.cycle_edges(5))
    with pytest.raises(ValueError):
        O.solve(prob, rank_test="lambda_max")
