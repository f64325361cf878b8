"""Pins for the oracle's PSD projections (Section 2.3.2 and Section 3.1).

Each check uses a fact fixed by the mathematics, not a retyped formula:
cone invariants, the Moreau decomposition S = proj(S) - proj(-S) of the
self-dual PSD cone, closed forms for diagonal and 2x2 inputs, and the
Eckart-Young characterisation of the truncated projection.
"""
import math

import numpy as np
import pytest

import instances as I
import oracle as O


def _rand_sym(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) * spread
    return 0.5 * (a + a.T)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (40, 3)])
def test_proj_cone_invariants(n, seed):
    S = _rand_sym(n, seed)
    P = O.proj_psd(S)
    scale = max(1.0, np.abs(S).max())
    assert np.allclose(P, P.T, atol=1e-13 * scale)
    assert np.linalg.eigvalsh(P)[0] >= -1e-12 * scale           # P is PSD
    assert np.allclose(O.proj_psd(P), P, atol=1e-11 * scale)      # idempotent
    assert abs(np.sum((S - P) * P)) <= 1e-10 * scale ** 2 * n      # <S-P, P> = 0
    assert np.linalg.eigvalsh(S - P)[-1] <= 1e-12 * scale         # S - P is NSD


@pytest.mark.parametrize("seed", range(4))
def test_proj_moreau_self_dual(seed):
    # PSD cone is self-dual: S = proj(S) - proj(-S) for every symmetric S
    S = _rand_sym(12, 10 + seed)
    assert np.allclose(S, O.proj_psd(S) - O.proj_psd(-S), atol=1e-12)


def test_proj_closed_forms():
    d = np.array([3.0, -1.0, 0.0, 2.5, -7.0])
    assert np.allclose(O.proj_psd(np.diag(d)), np.diag(np.maximum(d, 0)))
    assert np.allclose(O.proj_psd(-2.0 * np.eye(6)), 0.0)
    Z = np.array([[2.0, 1.0], [1.0, 3.0]])
    assert np.allclose(O.proj_psd(Z), Z)                           # PSD input unchanged


@pytest.mark.parametrize("a,b,c", [(1.0, 2.0, -1.0), (-3.0, 0.5, 1.0), (0.2, -4.0, 0.1),
                                   (-1.0, 0.1, -2.0), (2.0, 0.0, -5.0)])
def test_proj_2x2_closed_form(a, b, c):
    S = np.array([[a, b], [b, c]])
    mean = 0.5 * (a + c)
    rad = math.hypot(0.5 * (a - c), b)
    l1, l2 = mean + rad, mean - rad
    if l2 >= 0:
        want = S
    elif l1 <= 0:
        want = np.zeros((2, 2))
    else:
        v = np.array([b, l1 - a]) if abs(b) > 1e-15 else (np.array([1.0, 0.0]) if a >= c
                                                          else np.array([0.0, 1.0]))
        v = v / np.linalg.norm(v)
        want = l1 * np.outer(v, v)
    assert np.allclose(O.proj_psd(S), want, atol=1e-13)


def test_proj_is_nearest_psd_among_samples():
    S = _rand_sym(6, 99)
    P = O.proj_psd(S)
    rng = np.random.default_rng(5)
    best = np.linalg.norm(S - P)
    for _ in range(300):
        G = rng.standard_normal((6, 6))
        Z = P + 0.05 * (G @ G.T) if _ % 2 else O.proj_psd(P + 0.1 * _rand_sym(6, _))
        assert np.linalg.norm(S - Z) >= best - 1e-12


@pytest.mark.parametrize("n,r,seed", [(30, 1, 0), (30, 4, 1), (50, 8, 2), (17, 17, 3)])
def test_aproj_invariants(n, r, seed):
    S = _rand_sym(n, 20 + seed)
    P = O.aproj_psd(S, r)
    ev = np.linalg.eigvalsh(P)
    assert ev[0] >= -1e-12
    assert np.sum(ev > 1e-9) <= r                                  # rank <= r
    assert abs(np.sum((S - P) * P)) <= 1e-9                        # <S-P, P> = 0


@pytest.mark.parametrize("n,r,seed", [(25, 3, 0), (40, 6, 1), (40, 1, 2)])
def test_aproj_equals_proj_when_rank_suffices(n, r, seed):
    lam = np.concatenate([np.linspace(1.0, 9.0, r), -np.linspace(0.5, 3.0, n - r)])
    S = I.random_symmetric(n, lam, seed)
    assert np.allclose(O.aproj_psd(S, r), O.proj_psd(S), atol=1e-11)
    assert np.allclose(O.aproj_psd(S, r + 2), O.proj_psd(S), atol=1e-11)


@pytest.mark.parametrize("n,r,seed", [(30, 2, 0), (30, 5, 1), (60, 10, 2)])
def test_aproj_eckart_young_error(n, r, seed):
    # ||proj - aproj||_F^2 = sum_{i>r} max(lambda_i, 0)^2 (Section 3.1, read with squares)
    S = _rand_sym(n, 40 + seed)
    lam = np.sort(np.linalg.eigvalsh(S))[::-1]
    err2 = np.linalg.norm(O.proj_psd(S) - O.aproj_psd(S, r)) ** 2
    assert err2 == pytest.approx(np.sum(np.maximum(lam[r:], 0) ** 2), rel=1e-9, abs=1e-12)
    # bound (n - r) max(lambda_{r+1}, 0)^2 <= (n - r) max(lambda_r, 0)^2
    assert err2 <= (n - r) * max(lam[r], 0) ** 2 + 1e-12
    # distance to S: the kept part is exact, the rest is dropped
    d2 = np.linalg.norm(S - O.aproj_psd(S, r)) ** 2
    want = np.sum(lam[r:] ** 2) + np.sum(np.minimum(lam[:r], 0) ** 2)
    assert d2 == pytest.approx(want, rel=1e-9)


def test_aproj_diagonal_closed_form():
    d = np.array([0.5, 4.0, -2.0, 3.0, 1.0, -0.1])
    P = O.aproj_psd(np.diag(d), 2)
    assert np.allclose(P, np.diag([0, 4.0, 0, 3.0, 0, 0]))
    P = O.aproj_psd(np.diag(-np.abs(d)), 3)
    assert np.allclose(P, 0)


def test_aproj_best_psd_rank_r_among_samples():
    # aproj(S, r) is a nearest PSD matrix of rank <= r to S
    S = _rand_sym(8, 7)
    r = 3
    P = O.aproj_psd(S, r)
    best = np.linalg.norm(S - P)
    rng = np.random.default_rng(11)
    lam, U = np.linalg.eigh(P)
    V = U[:, -r:] * np.sqrt(np.maximum(lam[-r:], 0))
    for _ in range(400):
        W = V + 0.05 * rng.standard_normal(V.shape)
        assert np.linalg.norm(S - W @ W.T) >= best - 1e-12
