"""Pins for the oracle's constraint operators, step size and dual resolvent.

* A(X) is checked against tr(A_i X) computed from dense A_i built
  independently from the triplets (pins the doubled off-diagonal weight).
* The adjoint identity <M(X), y> = <X, M*(y)> (Section 1.3).
* ||M||_2 against closed forms and a dense SVD of the stacked vec(M_i).
* The dual resolvent of Section 2.3.1 against a direct numerical
  minimisation of the scalar proximal problem of the conjugate.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import instances as I
import oracle as O


def _dense_rows(prob):
    n = prob.n
    rows = [np.zeros((n, n)) for _ in range(prob.m + prob.p)]
    for r, i, j, v in zip(prob.a_row, prob.a_i, prob.a_j, prob.a_v):
        rows[r][i, j] += v
        if i != j:
            rows[r][j, i] += v
    for t, r in enumerate(prob.r1_row):
        u = prob.r1_u[t]
        rows[r] += prob.r1_sigma[t] * np.outer(u, u)
    return rows


def _small_general_problem(seed):
    rng = np.random.default_rng(seed)
    n = 6
    m, p = 3, 4
    ent = []
    for row in range(m + p):
        k = rng.integers(1, 5)
        for _ in range(k):
            i, j = sorted(rng.integers(0, n, 2))
            ent.append((row, i, j, rng.standard_normal()))
    ent.append((0, 1, 2, 0.7))   # duplicate entries are summed
    ent.append((0, 1, 2, 0.3))
    e = np.array(ent)
    prob = I.Problem(n=n, m=m, p=p, c_i=[0, 1, 2], c_j=[0, 3, 2], c_v=[1.0, -0.5, 2.0],
                     a_row=e[:, 0], a_i=e[:, 1], a_j=e[:, 2], a_v=e[:, 3],
                     b=rng.standard_normal(m), h=rng.standard_normal(p),
                     r1_row=[5], r1_sigma=[0.5], r1_u=rng.standard_normal((1, n)))
    return prob


@pytest.mark.parametrize("seed", range(3))
def test_apply_matches_dense_traces(seed):
    prob = _small_general_problem(seed)
    ops = O.Operators(prob, row_scaling=False)
    X = np.random.default_rng(seed).standard_normal((6, 6))
    X = X + X.T
    want = np.array([np.trace(Ai @ X) for Ai in _dense_rows(prob)])
    assert np.allclose(ops.apply(X), want, atol=1e-12)
    C = O.dense_sym_from_coo(6, prob.c_i, prob.c_j, prob.c_v)
    assert np.allclose(ops.C(), C)


@pytest.mark.parametrize("seed", range(3))
def test_adjointness(seed):
    prob = _small_general_problem(seed)
    for scaling in (False, True):
        ops = O.Operators(prob, row_scaling=scaling)
        rng = np.random.default_rng(100 + seed)
        X = rng.standard_normal((6, 6))
        X = X + X.T
        y = rng.standard_normal(prob.m + prob.p)
        assert np.dot(ops.apply(X), y) == pytest.approx(np.sum(X * ops.adjoint(y)), rel=1e-12)
        # adjoint equals sum_i y_i M_i built densely (row-scaled)
        Ms = _dense_rows(prob)
        want = sum(y[i] * Ms[i] / ops.scale[i] for i in range(len(Ms)))
        assert np.allclose(ops.adjoint(y), want, atol=1e-12)


def test_row_scaling_unit_frobenius():
    prob = _small_general_problem(4)
    ops = O.Operators(prob, row_scaling=True)
    Ms = _dense_rows(prob)
    for i, Mi in enumerate(Ms):
        assert ops.scale[i] == pytest.approx(np.linalg.norm(Mi), rel=1e-12)
    assert np.allclose(np.sqrt(np.asarray(ops.M.multiply(ops.M).sum(1)).ravel()), 1.0)


def test_norm_closed_forms():
    # max-cut: rows e_i e_i^T are orthonormal -> ||M|| = 1
    p = I.maxcut(30, 0.2, 0)
    assert O.Operators(p).norm() == pytest.approx(1.0, rel=1e-12)
    # equipartition with the all-ones row scaled to unit norm: sqrt(1 + 1/sqrt(n))
    for n in (9, 16, 40):
        p = I.equipartition(n, 0.3, 1)
        assert O.Operators(p).norm() == pytest.approx(math.sqrt(1 + 1 / math.sqrt(n)), rel=1e-10)


@pytest.mark.parametrize("seed", range(3))
def test_norm_matches_dense_svd(seed):
    prob = _small_general_problem(seed)
    ops = O.Operators(prob, row_scaling=False)
    stack = np.stack([Mi.ravel() for Mi in _dense_rows(prob)])
    assert ops.norm() == pytest.approx(np.linalg.svd(stack, compute_uv=False)[0], rel=1e-10)


@pytest.mark.parametrize("u,alpha,bb,hh", [(0.3, 0.9, 1.0, 2.0), (-2.0, 0.5, -1.0, 0.7),
                                            (5.0, 1.3, 0.2, 1.5), (0.1, 0.1, 3.0, -2.0)])
def test_dual_resolvent_is_prox_of_conjugate(u, alpha, bb, hh):
    # (I + alpha dI*)^{-1}(u) = argmin_z I*(z) + (z - u)^2 / (2 alpha).
    # {= b}: I*(z) = b z.   {<= h}: I*(z) = h z for z >= 0, +inf otherwise.
    got = O.dual_resolvent(np.array([u, u]), alpha, np.array([bb]), np.array([hh]))
    z_eq = minimize_scalar(lambda z: bb * z + (z - u) ** 2 / (2 * alpha)).x
    z_in = minimize_scalar(lambda z: hh * z + (z - u) ** 2 / (2 * alpha),
                           bounds=(0.0, 100.0), method="bounded", options={"xatol": 1e-12}).x
    assert got[0] == pytest.approx(z_eq, abs=1e-7)
    assert got[1] == pytest.approx(z_in, abs=1e-6)


def test_box_projection():
    u = np.array([5.0, -1.0, 3.0, 0.5])
    got = O.proj_box(u, np.array([1.0, 2.0]), np.array([1.0, 1.0]))
    assert np.allclose(got, [1.0, 2.0, 1.0, 0.5])


def test_svec_isometry():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((7, 7))
    A = A + A.T
    B = rng.standard_normal((7, 7))
    B = B + B.T
    assert np.dot(O.svec(A), O.svec(B)) == pytest.approx(np.sum(A * B), rel=1e-13)
    assert np.allclose(O.smat(O.svec(A), 7), A)
    iu, ju = np.triu_indices(7)
    assert np.array_equal(O.svec_index(7, iu, ju), np.arange(iu.size))
