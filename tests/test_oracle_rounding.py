"""Pins of the oracle's random-hyperplane rounding (Goemans-Williamson, cited
in the paper's Section 1.1) and of the arccos expectation it is judged by."""
import math

import numpy as np

import instances as I
import oracle as O


def _dense_C(prob):
    return O.dense_sym_from_coo(prob.n, prob.c_i, prob.c_j, prob.c_v)


def test_rank_one_bipartite_optimum_rounds_to_the_bipartition():
    # even cycle C_8: the max-cut relaxation's optimum is x x^T with x the
    # alternating signs (all 8 edges cut); every hyperplane gives +-x
    n = 8
    prob = I.from_edges_maxcut(n, I.cycle_edges(n))
    x = np.array([1.0 if i % 2 == 0 else -1.0 for i in range(n)])
    V = (x / math.sqrt(n)).reshape(n, 1)
    lam = np.array([float(n)])
    G = np.random.default_rng(0).standard_normal((16, 1))
    xs, vals = O.hyperplane_round(V, lam, _dense_C(prob), G)
    assert np.all(vals == -8.0)
    for t in range(16):
        assert np.array_equal(xs[t], x) or np.array_equal(xs[t], -x)


def test_values_are_minus_the_cut_and_at_most_the_max_cut():
    # <-L/4, x x^T> = -(number of edges with x_i != x_j), counted from the
    # edge list; no rounding beats the brute-force maximum cut
    n = 12
    edges = I.erdos_renyi_edges(n, 0.4, 3)
    prob = I.from_edges_maxcut(n, edges)
    rng = np.random.default_rng(1)
    V = np.linalg.qr(rng.standard_normal((n, 4)))[0]
    lam = np.array([5.0, 3.0, 2.0, 0.5])
    G = rng.standard_normal((64, 4))
    xs, vals = O.hyperplane_round(V, lam, _dense_C(prob), G)
    best = O.brute_force_maxcut(n, edges)
    for t in range(64):
        cut = int(np.sum(xs[t][edges[:, 0]] != xs[t][edges[:, 1]]))
        assert vals[t] == -cut
        assert cut <= best


def test_arccos_expectation_two_vectors():
    # two unit vectors at angle theta are separated with probability theta / pi
    for c in (-0.9, -0.3, 0.0, 0.5, 0.99):
        X = np.array([[1.0, c], [c, 1.0]])
        assert abs(O.gw_expected_cut(X, np.array([[0, 1]])) - math.acos(c) / math.pi) <= 1e-15


def test_mean_of_roundings_matches_expectation_and_gw_bound():
    # the SDP optimum of a small graph, factored X = V diag(lam) V^T: the mean
    # cut of 4000 hyperplanes matches sum arccos(X_ij) / pi within sampling
    # error, and that expectation is at least 0.878 of the SDP bound
    n = 14
    edges = I.erdos_renyi_edges(n, 0.35, 5)
    prob = I.from_edges_maxcut(n, edges)
    res = O.solve(prob, tol=1e-8, full_eig=True)
    lam, U = O.eig_desc(res.X)
    keep = lam > 1e-9
    V, lam = U[:, keep], lam[keep]
    G = np.random.default_rng(7).standard_normal((4000, lam.size))
    xs, vals = O.hyperplane_round(V, lam, _dense_C(prob), G)
    cuts = -vals
    expect = O.gw_expected_cut(res.X, edges)
    se = cuts.std() / math.sqrt(cuts.size)
    assert abs(cuts.mean() - expect) <= 4.0 * se
    assert expect >= 0.878 * (-res.obj)
    assert cuts.max() <= O.brute_force_maxcut(n, edges)
