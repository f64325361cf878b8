"""Sensor localisation with noisy distances (Section 5.2 with the +-10 % bands
and 5 % multiplicative noise): the band set is empty, proved by a Farkas
certificate read off the oracle's own PDHG iterates.

With C = 0 the PDHG dual iterates of an infeasible problem grow linearly;
their displacement d (per iteration) is a direction with d_G <= 0 (inequality
duals are <= 0 in the Section 1.3 sign), M*(d) <= 0 and b^T d_A + h^T d_G > 0.
For any feasible Z, <M*(d), Z> = d_A^T A(Z) + d_G^T G(Z) >= b^T d_A + h^T d_G
(d_G <= 0, G(Z) <= h) while <M*(d), Z> <= lambda_max(M*(d)) tr(Z), so a
direction with b^T d_A + h^T d_G > max(lambda_max, 0) tau, tau a bound on
tr(Z) over the feasible set, proves that the set is empty.  tau comes from
the rows themselves: with Y - X^T X PSD an anchor row bounds
sqrt(Y_jj) <= |a_k| + sqrt(h_up) and a sensor-pair row propagates
sqrt(Y_jj) <= sqrt(Y_ii) + sqrt(h_up) (shortest paths from the anchors).
Without noise the true positions satisfy every row (the set is not empty)."""
import numpy as np
import pytest

import instances as I
import oracle as O
from snl_farkas import farkas_check, trace_bound


def _oracle_duals(prob, K, L):
    ops = O.Operators(prob)
    alpha = 0.95 / ops.norm()
    n = prob.n
    X = np.zeros((n, n))
    y = np.zeros(prob.m + prob.p)
    C = ops.C()
    MX = None
    keep = {}
    for k in range(1, K + 1):
        out = O.pdhg_step(ops, C, X, y, n, alpha, MX)
        X, y, MX = out.X, out.y, out.MX
        if k in (K - L, K):
            keep[k] = y.copy()
    return ops, keep[K - L], keep[K], out


def test_noiseless_bands_hold_at_the_true_positions():
    prob, pos, anchors = I.snl(30, 1, noise=0.0, return_truth=True)
    n = prob.n
    Z = np.zeros((n, n))
    Z[:2, :2] = np.eye(2)
    Z[:2, 2:] = pos.T
    Z[2:, :2] = pos
    Z[2:, 2:] = pos @ pos.T
    ops = O.Operators(prob, row_scaling=False)
    MZ = ops.apply(Z)
    assert np.allclose(MZ[:prob.m], prob.b, atol=1e-12)
    assert np.all(MZ[prob.m:] <= prob.h + 1e-12)
    assert trace_bound(prob) >= np.trace(Z)


@pytest.mark.parametrize("seed,K,L", [(1, 6000, 2000), (2, 20000, 5000)])
def test_noisy_band_set_is_empty(seed, K, L):
    prob = I.snl(30, seed, noise=0.05)
    tau = trace_bound(prob)
    ops, y1, y2, out = _oracle_duals(prob, K, L)
    # the residuals stall while the duals run away
    assert np.linalg.norm(y2 - y1) > 0.2 * np.linalg.norm(y2)
    assert out.eps_p / (1 + ops.norm_C) > 1e-5
    value, lam_max, ok = farkas_check(ops, (y2 - y1) / L, tau)
    assert value > 0.0
    assert ok, (value, lam_max, tau)
