"""Farkas certificate of an empty sensor-localisation band set (shared by the
oracle test and the GPU test); see test_oracle_snl_infeasible.py."""
import heapq

import numpy as np


def row_entries(prob):
    rows = {}
    for r, i, j, v in zip(prob.a_row, prob.a_i, prob.a_j, prob.a_v):
        rows.setdefault(int(r), []).append((int(i), int(j), float(v)))
    return rows


def trace_bound(prob):
    """Upper bound of tr(Z) over the band set (2 + sum of the Y_jj bounds)."""
    d = 2
    n = prob.n
    rows = row_entries(prob)
    h = prob.h
    m = prob.m
    best = np.full(n, np.inf)     # bound on sqrt(Y_jj), index in Z
    adj = [[] for _ in range(n)]
    for t in range(prob.p):
        if h[t] <= 0.0:          # lower band rows carry no upper bound
            continue
        ent = rows[m + t]
        root = np.sqrt(h[t])
        diag = {(i, j): v for i, j, v in ent}
        if (0, 0) in diag:       # anchor row: |a_k|^2 Z00 + Y_jj - 2 a_k^T x_j
            jj = next(i for i, j, v in ent if i == j and i >= d)
            best[jj] = min(best[jj], np.sqrt(diag[(0, 0)]) + root)
        else:                    # sensor pair: Y_ii + Y_jj - 2 Y_ij
            gi, gj = sorted({i for i, j, v in ent if i == j})
            adj[gi].append((gj, root))
            adj[gj].append((gi, root))
    heap = [(b, j) for j, b in enumerate(best) if np.isfinite(b)]
    heapq.heapify(heap)
    while heap:
        b, j = heapq.heappop(heap)
        if b > best[j]:
            continue
        for k, w in adj[j]:
            if b + w < best[k]:
                best[k] = b + w
                heapq.heappush(heap, (best[k], k))
    ys = best[d:]
    assert np.all(np.isfinite(ys)), "a sensor is not connected to an anchor"
    return 2.0 + float(np.sum(ys ** 2))


def farkas_check(ops, d, tau):
    """(value, lambda_max) of the direction d (scaled problem), with d_G
    clipped to <= 0 so that it is a valid dual direction."""
    m = ops.m
    dd = np.concatenate([d[:m], np.minimum(d[m:], 0.0)])
    lam_max = float(np.linalg.eigvalsh(ops.adjoint(dd))[-1])
    value = float(ops.rhs @ dd)
    return value, lam_max, value > max(lam_max, 0.0) * tau
