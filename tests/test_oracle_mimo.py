"""Pins of the binary MIMO detection instances (Section 5.3) and of the
oracle on them: the cost matrix reproduces the least-squares objective, the
box rows read +-X_ij, and at high signal-to-noise ratio the relaxation
recovers the transmitted signal (the exactness the paper relies on)."""
import itertools

import numpy as np
import pytest

import instances as I
import oracle as O


def _L(prob):
    return O.dense_sym_from_coo(prob.n, prob.c_i, prob.c_j, prob.c_v)


def test_cost_is_the_least_squares_objective():
    n = 7
    prob = I.mimo(n, 3, sigma=0.3)
    H, x, y = I.mimo_signal(n, 3, 0.3)
    L = _L(prob)
    rng = np.random.default_rng(0)
    for _ in range(10):
        z = np.where(rng.random(n) < 0.5, -1.0, 1.0)
        zz = np.append(z, 1.0)
        assert zz @ L @ zz == pytest.approx(np.sum((H @ z - y) ** 2), rel=1e-12)
    assert np.linalg.eigvalsh(L)[0] >= -1e-9 * np.abs(L).max()   # L = [H, -y]^T [H, -y]


def test_box_rows_read_plus_minus_entries():
    n = 5
    prob = I.mimo(n, 1)
    ops = O.Operators(prob, row_scaling=False)
    rng = np.random.default_rng(2)
    A = rng.standard_normal((n + 1, n + 1))
    X = A + A.T
    MX = ops.apply(X)
    iu, ju = np.triu_indices(n + 1, 1)
    assert np.allclose(MX[:n + 1], np.diag(X))
    assert np.allclose(MX[n + 1::2], X[iu, ju])
    assert np.allclose(MX[n + 2::2], -X[iu, ju])
    assert np.all(prob.h == 1.0) and np.all(prob.b == 1.0)


def test_true_signal_is_feasible_and_optimal_without_noise():
    # y = H x: tr(L X) >= 0 for every PSD X and the lifted signal reaches 0
    n = 12
    prob = I.mimo(n, 5, sigma=0.0)
    x = prob.meta["x_true"]
    xx = np.append(x, 1.0)
    X = np.outer(xx, xx)
    ops = O.Operators(prob, row_scaling=False)
    MX = ops.apply(X)
    assert np.allclose(MX[:n + 1], 1.0) and np.all(MX[n + 1:] <= 1.0 + 1e-12)
    assert abs(np.sum(_L(prob) * X)) <= 1e-9 * np.abs(_L(prob)).max()


@pytest.mark.parametrize("n,seed", [(8, 0), (10, 4)])
def test_relaxation_recovers_the_maximum_likelihood_signal(n, seed):
    # high SNR: the relaxation's answer, read from its last column, is the
    # brute-force least-squares minimiser over {-1, +1}^n (and the signal)
    prob = I.mimo(n, seed, sigma=0.05)
    H, x, y = I.mimo_signal(n, seed, 0.05)
    best, arg = np.inf, None
    for bits in itertools.product((-1.0, 1.0), repeat=n):
        z = np.array(bits)
        v = np.sum((H @ z - y) ** 2)
        if v < best:
            best, arg = v, z
    res = O.solve(prob, tol=1e-6, full_eig=True, max_iters=200000)
    assert res.status == O.CONVERGED
    xhat = np.sign(res.X[:n, n])
    assert np.array_equal(xhat, arg) and np.array_equal(arg, x)
    # the relaxation bounds the least-squares value from below and is tight here
    assert res.obj <= best * (1 + 1e-3) + 1e-3
    assert res.obj >= best - 1e-3 * (1 + np.abs(_L(prob)).max())


def test_lr_solve_recovers_signal_at_n_100():
    n = 100
    prob = I.mimo(n, 1, sigma=0.1)
    res = O.solve(prob, tol=1e-4, max_iters=20000)
    assert res.status == O.CONVERGED
    assert np.array_equal(np.sign(res.X[:n, n]), prob.meta["x_true"])
    cert = O.certificate(prob, res.X, res.y)
    assert max(cert.rho_p, cert.rho_d) <= 2e-4
