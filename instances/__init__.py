"""Seeded synthetic SDP instances.

This module only *generates problem data*: the cost matrix C, the constraint
rows and their right-hand sides, in the layout of the library's C interface.
It holds none of the solver's arithmetic, so both the CPU oracle and the GPU
path may draw their inputs from it.

Problem form (general SDP form of Section 1.3 of the paper)::

    minimize  tr(C X)   s.t.  A(X) = b  (rows 0..m-1),
                              G(X) <= h (rows m..m+p-1),   X PSD, X in S^n.

Every symmetric matrix is given by its upper triangle (i <= j) as COO
triplets; an off-diagonal entry v at (i, j) stands for v at both (i, j) and
(j, i), so it contributes 2 v X_ij to tr(A X).  Duplicated triplets are summed.
A row may also carry rank-one terms sigma * u u^T (used for the all-ones
matrix of the graph-equipartition constraint, which would otherwise be n^2/2
triplets).

Workloads (recipes stated with each generator):

* ``maxcut``        -- Goemans-Williamson relaxation, C = -L/4, diag(X) = 1.
* ``equipartition`` -- Section 5.1: min <L, X>, diag(X) = 1, <11^T, X> = 0.
* ``snl``           -- Section 5.2: sensor network localisation with noisy
                       two-sided distance inequalities.
* ``mimo``          -- Section 5.3: binary MIMO detection, dense cost and
                       element-wise box inequalities.
* ``random_symmetric`` -- dense symmetric test matrices with a prescribed
                       spectrum, for the PSD-projection entry point.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem",
    "erdos_renyi_edges",
    "laplacian_coo",
    "maxcut",
    "equipartition",
    "snl",
    "random_symmetric",
    "cycle_edges",
    "complete_edges",
    "from_edges_maxcut",
    "from_edges_equipartition",
    "planted_lowrank",
    "mimo",
    "mimo_signal",
]


@dataclass
class Problem:
    """Problem data in the C-interface layout (all arrays host numpy)."""

    n: int
    m: int
    p: int
    c_i: np.ndarray
    c_j: np.ndarray
    c_v: np.ndarray
    a_row: np.ndarray
    a_i: np.ndarray
    a_j: np.ndarray
    a_v: np.ndarray
    b: np.ndarray
    h: np.ndarray
    r1_row: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    r1_sigma: np.ndarray = field(default_factory=lambda: np.zeros(0))
    r1_u: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.c_i = np.ascontiguousarray(self.c_i, dtype=np.int32)
        self.c_j = np.ascontiguousarray(self.c_j, dtype=np.int32)
        self.c_v = np.ascontiguousarray(self.c_v, dtype=np.float64)
        self.a_row = np.ascontiguousarray(self.a_row, dtype=np.int32)
        self.a_i = np.ascontiguousarray(self.a_i, dtype=np.int32)
        self.a_j = np.ascontiguousarray(self.a_j, dtype=np.int32)
        self.a_v = np.ascontiguousarray(self.a_v, dtype=np.float64)
        self.b = np.ascontiguousarray(self.b, dtype=np.float64).reshape(-1)
        self.h = np.ascontiguousarray(self.h, dtype=np.float64).reshape(-1)
        self.r1_row = np.ascontiguousarray(self.r1_row, dtype=np.int32).reshape(-1)
        self.r1_sigma = np.ascontiguousarray(self.r1_sigma, dtype=np.float64).reshape(-1)
        u = np.asarray(self.r1_u, dtype=np.float64)
        if u.size == 0:
            u = np.zeros((0, self.n))
        self.r1_u = np.ascontiguousarray(u.reshape(-1, self.n))
        assert self.b.shape == (self.m,) and self.h.shape == (self.p,)

    @property
    def n_rows(self) -> int:
        return self.m + self.p


# --------------------------------------------------------------------- graphs
def erdos_renyi_edges(n: int, p_edge: float, seed: int) -> np.ndarray:
    """G(n, p): each pair i < j is an edge independently with probability p.

    One uniform draw per upper-triangle pair, in row-major order, from a PCG64
    stream seeded with ``seed``.  Returns an (E, 2) int32 array with i < j.
    """
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p_edge
    return np.stack([iu[keep], ju[keep]], axis=1).astype(np.int32)


def cycle_edges(n: int) -> np.ndarray:
    i = np.arange(n)
    e = np.stack([i, (i + 1) % n], axis=1)
    return np.sort(e, axis=1).astype(np.int32)


def complete_edges(n: int) -> np.ndarray:
    iu, ju = np.triu_indices(n, 1)
    return np.stack([iu, ju], axis=1).astype(np.int32)


def laplacian_coo(n: int, edges: np.ndarray, weights: np.ndarray | None = None):
    """Upper-triangle COO of the weighted graph Laplacian L = D - W."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.ones(e.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64)
    deg = np.zeros(n)
    np.add.at(deg, e[:, 0], w)
    np.add.at(deg, e[:, 1], w)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    ii = np.concatenate([np.arange(n), lo])
    jj = np.concatenate([np.arange(n), hi])
    vv = np.concatenate([deg, -w])
    return ii.astype(np.int32), jj.astype(np.int32), vv


def _diag_rows(n: int):
    r = np.arange(n, dtype=np.int32)
    return r, r.copy(), r.copy(), np.ones(n)


def from_edges_maxcut(n: int, edges: np.ndarray, name: str = "maxcut", meta=None) -> Problem:
    """Max-cut relaxation: minimize <-L/4, X> s.t. X_ii = 1, X PSD.

    -<C, x x^T> equals the cut weight of x in {-1,1}^n, so the optimal value
    is minus the SDP upper bound on the maximum cut.
    """
    li, lj, lv = laplacian_coo(n, edges)
    a_row, a_i, a_j, a_v = _diag_rows(n)
    return Problem(n=n, m=n, p=0, c_i=li, c_j=lj, c_v=-0.25 * lv,
                   a_row=a_row, a_i=a_i, a_j=a_j, a_v=a_v,
                   b=np.ones(n), h=np.zeros(0), name=name,
                   meta=dict(meta or {}, edges=int(len(edges))))


def from_edges_equipartition(n: int, edges: np.ndarray, name: str = "equipartition",
                             meta=None) -> Problem:
    """Graph equipartition relaxation (Section 5.1):

    minimize <L, X> s.t. X_ii = 1 (rows 0..n-1), <1 1^T, X> = 0 (row n), X PSD.
    The all-ones row is passed as one rank-one term (sigma = 1, u = 1).
    """
    li, lj, lv = laplacian_coo(n, edges)
    a_row, a_i, a_j, a_v = _diag_rows(n)
    return Problem(n=n, m=n + 1, p=0, c_i=li, c_j=lj, c_v=lv,
                   a_row=a_row, a_i=a_i, a_j=a_j, a_v=a_v,
                   b=np.concatenate([np.ones(n), [0.0]]), h=np.zeros(0),
                   r1_row=np.array([n], np.int32), r1_sigma=np.array([1.0]),
                   r1_u=np.ones((1, n)), name=name,
                   meta=dict(meta or {}, edges=int(len(edges))))


def maxcut(n: int, p_edge: float, seed: int) -> Problem:
    """Max-cut on G(n, p_edge) with unit weights (C = -L/4, diag(X) = 1)."""
    return from_edges_maxcut(n, erdos_renyi_edges(n, p_edge, seed),
                             name=f"maxcut_n{n}_p{p_edge}_s{seed}",
                             meta=dict(kind="maxcut", p_edge=p_edge, seed=seed))


def equipartition(n: int, p_edge: float, seed: int) -> Problem:
    """Graph equipartition on G(n, p_edge) with unit weights."""
    return from_edges_equipartition(n, erdos_renyi_edges(n, p_edge, seed),
                                    name=f"equip_n{n}_p{p_edge}_s{seed}",
                                    meta=dict(kind="equipartition", p_edge=p_edge, seed=seed))


def planted_lowrank(n: int, rank: int, seed: int) -> Problem:
    """Diagonal-constrained SDP with a dense rank-``rank`` cost (a test case
    with a planted spectral gap): minimize <C, X> s.t. X_ii = 1, X PSD, with
    C = -U diag(s) U^T, U an n x rank Haar-orthonormal block (QR of a PCG64
    Gaussian matrix seeded with ``seed``) and s spaced evenly from 2 n / rank
    down to n / rank.  The first iterates W = -alpha C have exactly ``rank``
    positive eigenvalues and a zero bulk, so a partial eigensolve of width
    k >= rank converges in a few rounds.  C is passed as its full upper
    triangle (n (n + 1) / 2 triplets).
    """
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, rank)))
    s = np.linspace(2.0, 1.0, rank) * (n / rank)
    C = -(U * s) @ U.T
    iu, ju = np.triu_indices(n)
    a_row, a_i, a_j, a_v = _diag_rows(n)
    return Problem(n=n, m=n, p=0, c_i=iu, c_j=ju, c_v=C[iu, ju],
                   a_row=a_row, a_i=a_i, a_j=a_j, a_v=a_v, b=np.ones(n), h=np.zeros(0),
                   name=f"planted_n{n}_r{rank}_s{seed}",
                   meta=dict(kind="planted_lowrank", rank=rank, seed=seed))


# ------------------------------------------------------------------------ SNL
def snl(n_sensors: int, seed: int, radius: float = 0.3, noise: float = 0.05,
        band: float = 0.1, d: int = 2, return_truth: bool = False):
    """Sensor network localisation (Section 5.2) with noisy inequalities.

    Recipe: sensors uniform in [-0.5, 0.5]^2, anchors at the four corners
    (+-0.5, +-0.5).  A sensor pair or anchor-sensor pair is measured when its
    true distance is <= ``radius``; the measurement is
    d~ = d (1 + noise * xi), xi ~ N(0, 1).  The PSD variable is
    Z = [[I_d, X], [X^T, Y]] in S^{d+n}.  Rows:

    * 3 equalities pinning Z[0:2, 0:2] = I (Z00 = 1, Z11 = 1, Z01 = 0);
    * per sensor pair (i, j): E^(ij) placed on the Y block (offset d),
      two inequalities  <E, Z> <= (1+band) d~^2  and  -<E, Z> <= -(1-band) d~^2;
    * per anchor pair (k, j): U^(kj) with U_00 = a_k^T a_k, U_{d+j,d+j} = 1,
      U_{0:d, d+j} = -a_k (valid because Z00 = 1 is enforced), same two
      inequalities.

    C = 0 (a feasibility problem).
    """
    assert d == 2
    rng = np.random.default_rng(seed)
    pos = rng.random((n_sensors, 2)) - 0.5
    anchors = np.array([[-0.5, -0.5], [-0.5, 0.5], [0.5, -0.5], [0.5, 0.5]])
    N = d + n_sensors
    # sensor pairs, by rows of the upper triangle, to bound memory
    si, sj = [], []
    for i in range(n_sensors - 1):
        dd = np.sqrt(((pos[i + 1:] - pos[i]) ** 2).sum(1))
        j = np.nonzero(dd <= radius)[0] + i + 1
        si.append(np.full(j.shape, i))
        sj.append(j)
    si = np.concatenate(si) if si else np.zeros(0, np.int64)
    sj = np.concatenate(sj) if sj else np.zeros(0, np.int64)
    ds = np.sqrt(((pos[si] - pos[sj]) ** 2).sum(1))
    ds_noisy = ds * (1.0 + noise * rng.standard_normal(ds.shape[0]))
    ak, aj = [], []
    for k in range(anchors.shape[0]):
        dd = np.sqrt(((pos - anchors[k]) ** 2).sum(1))
        j = np.nonzero(dd <= radius)[0]
        ak.append(np.full(j.shape, k))
        aj.append(j)
    ak = np.concatenate(ak)
    aj = np.concatenate(aj)
    da = np.sqrt(((pos[aj] - anchors[ak]) ** 2).sum(1))
    da_noisy = da * (1.0 + noise * rng.standard_normal(da.shape[0]))

    rows_r, rows_i, rows_j, rows_v = [], [], [], []
    # equalities 0..2
    rows_r += [0, 1, 2]
    rows_i += [0, 1, 0]
    rows_j += [0, 1, 1]
    rows_v += [1.0, 1.0, 0.5]
    b = np.array([1.0, 1.0, 0.0])
    m = 3
    ns = si.shape[0]
    na = ak.shape[0]
    # sensor pair rows: row index m + 2q (upper) and m + 2q + 1 (lower)
    q = np.arange(ns)
    r_up = m + 2 * q
    r_lo = r_up + 1
    gi, gj = d + si, d + sj
    sens_r = np.concatenate([r_up, r_up, r_up, r_lo, r_lo, r_lo])
    sens_i = np.concatenate([gi, gj, gi, gi, gj, gi])
    sens_j = np.concatenate([gi, gj, gj, gi, gj, gj])
    one = np.ones(ns)
    sens_v = np.concatenate([one, one, -one, -one, -one, one])
    h_s = np.empty(2 * ns)
    h_s[0::2] = (1.0 + band) * ds_noisy ** 2
    h_s[1::2] = -(1.0 - band) * ds_noisy ** 2
    # anchor rows
    qa = np.arange(na)
    ra_up = m + 2 * ns + 2 * qa
    ra_lo = ra_up + 1
    a = anchors[ak]
    jj = d + aj
    anc_r, anc_i, anc_j, anc_v = [], [], [], []
    for sgn, rr in ((1.0, ra_up), (-1.0, ra_lo)):
        anc_r += [rr, rr, rr, rr]
        anc_i += [np.zeros(na, np.int64), jj, np.zeros(na, np.int64), np.ones(na, np.int64)]
        anc_j += [np.zeros(na, np.int64), jj, jj, jj]
        anc_v += [sgn * (a ** 2).sum(1), sgn * np.ones(na), -sgn * a[:, 0], -sgn * a[:, 1]]
    h_a = np.empty(2 * na)
    h_a[0::2] = (1.0 + band) * da_noisy ** 2
    h_a[1::2] = -(1.0 - band) * da_noisy ** 2

    a_row = np.concatenate([np.array(rows_r), sens_r, np.concatenate(anc_r)])
    a_i = np.concatenate([np.array(rows_i), sens_i, np.concatenate(anc_i)])
    a_j = np.concatenate([np.array(rows_j), sens_j, np.concatenate(anc_j)])
    a_v = np.concatenate([np.array(rows_v), sens_v, np.concatenate(anc_v)])
    prob = Problem(n=N, m=m, p=2 * (ns + na),
                   c_i=np.zeros(0), c_j=np.zeros(0), c_v=np.zeros(0),
                   a_row=a_row, a_i=a_i, a_j=a_j, a_v=a_v,
                   b=b, h=np.concatenate([h_s, h_a]),
                   name=f"snl_n{n_sensors}_s{seed}",
                   meta=dict(kind="snl", sensors=n_sensors, seed=seed, radius=radius,
                             noise=noise, band=band, sensor_pairs=int(ns),
                             anchor_pairs=int(na)))
    if return_truth:
        return prob, pos, anchors
    return prob


# ----------------------------------------------------------------------- MIMO
def mimo_signal(n: int, seed: int, sigma: float = 0.1):
    """Channel, signal and received vector of a binary MIMO instance
    (Section 5.3): H is n x n with i.i.d. N(0, 1) entries, x in {-1, +1}^n
    uniform, y = H x + sigma * eps with eps ~ N(0, I).  One PCG64 stream seeded
    with ``seed``, drawn in the order H (row-major), x, eps."""
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((n, n))
    x = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    y = H @ x + sigma * rng.standard_normal(n)
    return H, x, y


def mimo(n: int, seed: int, sigma: float = 0.1) -> Problem:
    """Binary MIMO detection relaxation (Section 5.3) on X in S^(n+1):

        minimize tr(L X)  s.t.  X_ii = 1 (i = 0..n),  -1 <= X_ij <= 1 (i < j),  X PSD,

    L = [[H^T H, -H^T y], [-y^T H, y^T y]], so that for x in {-1, +1}^n,
    [x; 1]^T L [x; 1] = ||H x - y||^2.  C = L is dense (all (n+1)(n+2)/2
    upper-triangle triplets).  Each off-diagonal pair (i, j), in row-major
    order of the upper triangle, gives two inequality rows: X_ij <= 1 (row
    n + 1 + 2q, triplet (i, j, 1/2)) and -X_ij <= 1 (row n + 2 + 2q, triplet
    (i, j, -1/2)); the diagonal is fixed by the equalities, so its box rows
    are left out.  At high signal-to-noise ratio the relaxation is exact: the
    optimum is X = [x; 1][x; 1]^T with x the transmitted signal.
    """
    H, x, y = mimo_signal(n, seed, sigma)
    N = n + 1
    L = np.zeros((N, N))
    L[:n, :n] = H.T @ H
    L[:n, n] = -H.T @ y
    L[n, :n] = L[:n, n]
    L[n, n] = y @ y
    iu, ju = np.triu_indices(N)
    a_row0, a_i0, a_j0, a_v0 = _diag_rows(N)
    ou, ov = np.triu_indices(N, 1)
    q = np.arange(ou.size)
    r_up = N + 2 * q
    a_row = np.concatenate([a_row0, r_up, r_up + 1])
    a_i = np.concatenate([a_i0, ou, ou])
    a_j = np.concatenate([a_j0, ov, ov])
    a_v = np.concatenate([a_v0, np.full(ou.size, 0.5), np.full(ou.size, -0.5)])
    return Problem(n=N, m=N, p=2 * ou.size, c_i=iu, c_j=ju, c_v=L[iu, ju],
                   a_row=a_row, a_i=a_i, a_j=a_j, a_v=a_v,
                   b=np.ones(N), h=np.ones(2 * ou.size),
                   name=f"mimo_n{n}_s{seed}",
                   meta=dict(kind="mimo", n_signal=n, seed=seed, sigma=sigma, x_true=x))


# ------------------------------------------------------ dense test matrices
def random_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix (QR of a Gaussian, sign-fixed)."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))


def random_symmetric(n: int, eigenvalues, seed: int) -> np.ndarray:
    """Dense symmetric U diag(eigenvalues) U^T with U Haar-orthogonal."""
    rng = np.random.default_rng(seed)
    lam = np.asarray(eigenvalues, dtype=np.float64)
    assert lam.shape == (n,)
    u = random_orthogonal(n, rng)
    s = (u * lam) @ u.T
    return 0.5 * (s + s.T)


def lowrank_plus_negative_spectrum(n: int, r_pos: int, seed: int, top: float = 100.0,
                                   gap: float = 10.0, neg: float = 20.0) -> np.ndarray:
    """Spectrum shaped like a PDHG iterate W = X - alpha*S near the optimum:
    ``r_pos`` positive eigenvalues in [gap, top] and n - r_pos values in
    [-neg, 0].  Returns the eigenvalues (not sorted)."""
    rng = np.random.default_rng(seed + 7919)
    pos = gap + (top - gap) * rng.random(r_pos)
    rest = -neg * rng.random(n - r_pos)
    return np.concatenate([pos, rest])


def serving_stream(count: int, seed: int = 0, n_lo: int = 100, n_hi: int = 2000,
                   mean_degree: float = 8.0, rate: float | None = None):
    """The serving workload: `count` requests, request i is max-cut or
    equipartition (one fair coin) on G(n, mean_degree / n) with n uniform in
    {n_lo .. n_hi}, graph seed = i.  Arrivals form a Poisson process of the
    given rate (requests per second; None = all at time 0).

    Returns a list of (request id, arrival time in s, Problem).
    """
    rng = np.random.default_rng(seed)
    kinds = rng.integers(0, 2, size=count)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    if rate is None:
        arrivals = np.zeros(count)
    else:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        n = int(sizes[i])
        p_edge = min(1.0, mean_degree / n)
        prob = maxcut(n, p_edge, i) if kinds[i] == 0 else equipartition(n, p_edge, i)
        out.append((i, float(arrivals[i]), prob))
    return out
