"""Plain FP64 CPU oracle for PD-SDP / LR-PD-SDP (Souto, Garcia, Veiga,
"Exploiting Low-Rank Structure in Semidefinite Programming by Approximate
Operator Splitting", arXiv 1810.05231).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library shares
no code with it.

Everything here is float64 NumPy/SciPy, with a full symmetric
eigendecomposition (LAPACK, ``numpy.linalg.eigh``) in every iteration.  The
functions follow the paper's order and notation; where the paper is silent
or inconsistent the reading taken is stated in the docstring (R-labels):

R1  Dual sign (Section 1.3 dual problem vs Algorithm 1).  The iterate ``y``
    is the dual variable of the dual problem in Section 1.3, i.e. the
    negative of Algorithm 1's y.  The primal step then reads
    X+ = proj(X - alpha (C - M*(y))), equality duals move by
    +alpha (b - A(Xbar)) and inequality duals are clamped to <= 0.
R2  Row scaling.  Each constraint row M_i (and b_i / h_i) is divided by its
    Frobenius norm before iterating; the step is alpha = 0.95 / ||M||_2 of
    the scaled operator (Section 2.2 only bounds alpha < 1/||M||_2).
    Returned duals are unscaled.  Residuals are those of the scaled
    iteration.
R3  Relative stopping rule.  rho_p = eps_primal / (1 + ||C||_F),
    rho_d = eps_dual / (1 + ||[b; h]||_2) with eps as in Section 2.2 (sign
    per R1); stop when max(rho_p, rho_d) <= tol.
R4  Control of Algorithm 2.  Tests run every ``check_every`` iterations.
    The window test compares eps_comb now with eps_comb ell iterations ago,
    counting only iterations after the last rank change.  Convergence
    requires the residual test AND the rank test (n - r) max(lambda_r, 0)
    <= eps_lambda (default eps_lambda = tol); a converged iterate that fails
    the rank test is saved as X_[r] and r doubles; a stalled window doubles
    r.  At r = n the method is PD-SDP (Algorithm 1).
R5  X0 = 0, y0 = 0.
R6  aproj takes the r algebraically largest eigenvalues (Section 3.1).
R7  The truncation error identity of Section 3.1 is read with squares
    (Eckart-Young): ||proj - aproj||_F^2 = sum_{i>r} max(lambda_i, 0)^2.
R8  Rank cap.  Algorithm 2 doubles r until, at worst, r = n.  With a cap
    r_max < n the doubling is impossible once r = r_max: a converged iterate
    that fails the rank test there stops with status RANK_LIMIT (it is the
    feasible X_[r] of Section 3.2, not an optimum); a stalled window at the
    cap keeps iterating.  r_max = n (the default) is Algorithm 2 itself.
R9  Rank test variable.  The default is Algorithm 2's lambda_r (the r-th
    largest eigenvalue of the projected matrix).  rank_test="lambda_r_plus_1"
    uses the first excluded eigenvalue lambda_{r+1} instead (the quantity the
    Section 3.1 error bound is really about); r = n passes either way.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

SQRT2 = math.sqrt(2.0)

CONVERGED, MAX_ITERS, TIME_LIMIT, NUMERICAL, RANK_LIMIT = 0, 1, 2, 3, 4
STATUS_NAMES = {CONVERGED: "converged", MAX_ITERS: "max_iters",
                TIME_LIMIT: "time_limit", NUMERICAL: "numerical", RANK_LIMIT: "rank_limit"}
RANK_TESTS = ("lambda_r", "lambda_r_plus_1")


# ------------------------------------------------------------ svec geometry
def svec_index(n: int, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """Position of (i, j), i <= j, in the row-major upper triangle."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return i * n - (i * (i - 1)) // 2 + (j - i)


def svec(X: np.ndarray) -> np.ndarray:
    """Isometric vectorisation of a symmetric matrix: <A, X> = svec(A).svec(X)."""
    n = X.shape[0]
    iu, ju = np.triu_indices(n)
    w = np.where(iu == ju, 1.0, SQRT2)
    return X[iu, ju] * w


def smat(v: np.ndarray, n: int) -> np.ndarray:
    """Inverse of svec."""
    iu, ju = np.triu_indices(n)
    w = np.where(iu == ju, 1.0, 1.0 / SQRT2)
    X = np.zeros((n, n))
    X[iu, ju] = v * w
    X[ju, iu] = v * w
    return X


def dense_sym_from_coo(n: int, i, j, v) -> np.ndarray:
    """Symmetric matrix from upper-triangle triplets (duplicates summed)."""
    S = np.zeros((n, n))
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    v = np.asarray(v, dtype=np.float64)
    np.add.at(S, (i, j), v)
    off = i != j
    np.add.at(S, (j[off], i[off]), v[off])
    return S


# ---------------------------------------------------------------- operators
class Operators:
    """The stacked constraint operator M = [A; G] of Section 2 in svec form.

    Row i of ``Msv`` is svec(M_i); then M(X) = Msv @ svec(X) and
    M*(y) = smat(Msv^T y) (the adjoint sum_i y_i M_i of Section 1.3).
    """

    def __init__(self, prob, row_scaling: bool = True):
        n = prob.n
        self.n = n
        self.m = prob.m
        self.p = prob.p
        rows = prob.m + prob.p
        N = n * (n + 1) // 2
        self.N = N
        if np.any(prob.a_i > prob.a_j) or np.any(prob.c_i > prob.c_j):
            raise ValueError("entries must be upper-triangle (i <= j)")
        col = svec_index(n, prob.a_i, prob.a_j)
        val = prob.a_v * np.where(prob.a_i == prob.a_j, 1.0, SQRT2)
        M = sp.csr_matrix((val, (prob.a_row.astype(np.int64), col)), shape=(rows, N))
        M.sum_duplicates()
        if prob.r1_row.size:
            iu, ju = np.triu_indices(n)
            w = np.where(iu == ju, 1.0, SQRT2)
            add = []
            for t in range(prob.r1_row.size):
                u = prob.r1_u[t]
                dense = prob.r1_sigma[t] * u[iu] * u[ju] * w
                nz = np.nonzero(dense)[0]
                add.append(sp.csr_matrix((dense[nz], (np.full(nz.size, prob.r1_row[t]), nz)),
                                         shape=(rows, N)))
            M = (M + sum(add[1:], add[0])).tocsr()
            M.sum_duplicates()
        cvec = np.zeros(N)
        ccol = svec_index(n, prob.c_i, prob.c_j)
        np.add.at(cvec, ccol, prob.c_v * np.where(prob.c_i == prob.c_j, 1.0, SQRT2))
        self.c = cvec
        rhs = np.concatenate([prob.b, prob.h])
        norms = np.sqrt(np.asarray(M.multiply(M).sum(axis=1)).ravel())
        if row_scaling:
            if np.any(norms == 0):
                raise ValueError("a constraint row is identically zero")
            scale = norms
        else:
            scale = np.ones(rows)
        self.scale = scale
        self.M = sp.diags(1.0 / scale) @ M
        self.M = self.M.tocsr()
        self.Mt = self.M.T.tocsr()
        self.rhs = rhs / scale          # [b; h] of the scaled problem
        self.norm_C = float(np.linalg.norm(cvec))
        self.norm_rhs = float(np.linalg.norm(self.rhs))
        self._norm_M = None

    # M(X) and M*(y)
    def apply(self, X: np.ndarray) -> np.ndarray:
        return self.M @ svec(X)

    def adjoint(self, y: np.ndarray) -> np.ndarray:
        return smat(self.Mt @ y, self.n)

    def C(self) -> np.ndarray:
        return smat(self.c, self.n)

    def norm(self) -> float:
        """||M||_2 = largest singular value of the stacked operator."""
        if self._norm_M is None:
            rows = self.m + self.p
            if rows <= 3000:
                K = (self.M @ self.Mt).toarray()
                self._norm_M = float(math.sqrt(max(np.linalg.eigvalsh(K)[-1], 0.0)))
            else:
                op = spla.LinearOperator((rows, rows), matvec=lambda y: self.M @ (self.Mt @ y),
                                         dtype=np.float64)
                ev = spla.eigsh(op, k=1, which="LA", tol=1e-10, return_eigenvectors=False,
                                v0=np.ones(rows))
                self._norm_M = float(math.sqrt(ev[0]))
        return self._norm_M


# ------------------------------------------------------- projections (3.x)
def eig_desc(S: np.ndarray):
    """Full eigendecomposition, eigenvalues in decreasing order."""
    lam, U = np.linalg.eigh(S)
    return lam[::-1].copy(), U[:, ::-1].copy()


def proj_psd(S: np.ndarray) -> np.ndarray:
    """Euclidean projection onto the PSD cone (Section 2.3.2):
    sum_i max(0, lambda_i) u_i u_i^T."""
    lam, U = eig_desc(S)
    lp = np.maximum(lam, 0.0)
    return (U * lp) @ U.T


def aproj_psd(S: np.ndarray, r: int, return_eig: bool = False):
    """Truncated projection aproj(S, r) of Section 3.1 (reading R6):
    sum_{i<=r} max(0, lambda_i) u_i u_i^T over the r algebraically largest
    eigenvalues."""
    n = S.shape[0]
    r = min(max(int(r), 0), n)
    lam, U = eig_desc(S)
    lp = np.maximum(lam[:r], 0.0)
    P = (U[:, :r] * lp) @ U[:, :r].T
    if return_eig:
        return P, lam, U
    return P


def proj_box(u: np.ndarray, b: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Projection onto {u1 = b, u2 <= h} (Section 2.3.1)."""
    m = b.shape[0]
    return np.concatenate([b, np.minimum(u[m:], h)])


def dual_resolvent(u: np.ndarray, alpha: float, b: np.ndarray, h: np.ndarray) -> np.ndarray:
    """(I + alpha dI*)^{-1}(u) = u - alpha proj(u / alpha), via the extended
    Moreau decomposition (Section 2.3.1).  Written in Algorithm 1's sign."""
    return u - alpha * proj_box(u / alpha, b, h)


# ------------------------------------------------------------------ PDHG
@dataclass
class StepOut:
    X: np.ndarray
    y: np.ndarray
    lam: np.ndarray          # eigenvalues of W, decreasing
    eps_p: float
    eps_d: float
    MX: np.ndarray           # M(X+)


def pdhg_step(ops: Operators, C: np.ndarray, X: np.ndarray, y: np.ndarray, r: int,
              alpha: float, MX_prev: np.ndarray | None = None) -> StepOut:
    """One iteration of Algorithm 1 (r = n) or Algorithm 2's inner loop.

    Sign per R1: y is the Section 1.3 dual, y_alg1 = -y.
    """
    n = ops.n
    m = ops.m
    # primal step: X+ = aproj(X - alpha (M*(y_alg1) + C), r)
    W = X - alpha * (C - ops.adjoint(y))
    lam, U = eig_desc(W)
    rr = min(r, n)
    lp = np.maximum(lam[:rr], 0.0)
    Xn = (U[:, :rr] * lp) @ U[:, :rr].T
    # dual step part 1, in Algorithm 1's sign: y_half = y_alg1 + alpha M(2X+ - X)
    MXn = ops.apply(Xn)
    MX = ops.apply(X) if MX_prev is None else MX_prev
    y_alg1 = -y
    y_half = y_alg1 + alpha * (2.0 * MXn - MX)
    # dual step part 2: y+ = y_half - alpha proj(y_half / alpha)
    y_alg1_new = dual_resolvent(y_half, alpha, ops.rhs[:m], ops.rhs[m:])
    yn = -y_alg1_new
    # residuals of Section 2.2 in the sign of R1
    dX = Xn - X
    dy = yn - y
    eps_p = float(np.linalg.norm(dX / alpha + ops.adjoint(dy)))
    eps_d = float(np.linalg.norm(dy / alpha + (MXn - MX)))
    return StepOut(Xn, yn, lam, eps_p, eps_d, MXn)


@dataclass
class SolveResult:
    X: np.ndarray
    y: np.ndarray             # unscaled dual, Section 1.3 sign
    status: int
    iters: int
    r: int
    obj: float
    dual_obj: float
    rho_p: float
    rho_d: float
    eps_p: float
    eps_d: float
    lam_r: float
    alpha: float
    rank_path: list = field(default_factory=list)
    saved: list = field(default_factory=list)   # intermediate (iter, r, X_[r], y_[r]), y unscaled
    trace: list = field(default_factory=list)
    time_s: float = 0.0


def solve(prob, tol: float = 1e-4, r0: int = 1, full_eig: bool = False, window: int = 50,
          check_every: int = 10, max_iters: int = 100000, eps_lambda: float | None = None,
          alpha: float | None = None, row_scaling: bool = True, r_max: int | None = None,
          time_limit: float = float("inf"), X0=None, y0=None, keep_trace: bool = False,
          ops: Operators | None = None, rank_test: str = "lambda_r") -> SolveResult:
    """LR-PD-SDP (Algorithm 2) with PD-SDP (Algorithm 1) as the r = n case.

    Control per R3/R4/R8/R9; X0 = y0 = 0 unless given (R5).  ``y0`` is in
    the scaled space of R2.
    """
    if rank_test not in RANK_TESTS:
        raise ValueError(f"rank_test must be one of {RANK_TESTS}")
    t0 = time.perf_counter()
    if ops is None:
        ops = Operators(prob, row_scaling=row_scaling)
    n = ops.n
    if window % check_every != 0:
        raise ValueError("window must be a multiple of check_every")
    alpha = 0.95 / ops.norm() if alpha is None else float(alpha)
    eps_lambda = tol if eps_lambda is None else eps_lambda
    r_max = n if r_max is None else min(r_max, n)
    C = ops.C()
    X = np.zeros((n, n)) if X0 is None else np.array(X0, dtype=np.float64)
    y = np.zeros(ops.m + ops.p) if y0 is None else np.array(y0, dtype=np.float64)
    r = n if full_eig else min(max(r0, 1), r_max)
    MX = ops.apply(X)
    hist = []            # eps_comb at check points since the last rank change
    L = window // check_every
    status = MAX_ITERS
    rank_path = [(0, r)]
    saved = []
    trace = []
    out = None
    k = 0
    rho_p = rho_d = math.inf
    for k in range(1, max_iters + 1):
        out = pdhg_step(ops, C, X, y, r, alpha, MX)
        X, y, MX = out.X, out.y, out.MX
        if not (np.isfinite(out.eps_p) and np.isfinite(out.eps_d)):
            status = NUMERICAL
            break
        if k % check_every:
            continue
        rho_p = out.eps_p / (1.0 + ops.norm_C)
        rho_d = out.eps_d / (1.0 + ops.norm_rhs)
        lam_r = out.lam[r - 1] if r <= n else -math.inf
        if keep_trace:
            trace.append((k, r, rho_p, rho_d, float(lam_r)))
        if max(rho_p, rho_d) <= tol:
            if rank_test == "lambda_r":
                lam_test = lam_r
            else:
                lam_test = out.lam[r] if r < n else -math.inf
            if r >= n or (n - r) * max(lam_test, 0.0) <= eps_lambda:
                status = CONVERGED
                break
            saved.append((k, r, X.copy(), y / ops.scale))
            if r >= r_max:
                # the doubling of Algorithm 2 is impossible at the cap (R8)
                status = RANK_LIMIT
                break
            r = min(2 * r, r_max)
            rank_path.append((k, r))
            hist = []
            continue
        hist.append(out.eps_p + out.eps_d)
        if r < r_max and len(hist) > L and hist[-1] >= hist[-1 - L]:
            r = min(2 * r, r_max)
            rank_path.append((k, r))
            hist = []
        if time.perf_counter() - t0 > time_limit:
            status = TIME_LIMIT
            break
    y_unscaled = y / ops.scale
    obj = float(ops.c @ svec(X))
    dual_obj = float(ops.rhs @ y)
    lam_r = float(out.lam[min(r, n) - 1]) if out is not None else math.nan
    return SolveResult(X=X, y=y_unscaled, status=status, iters=k, r=r, obj=obj,
                       dual_obj=dual_obj, rho_p=float(rho_p), rho_d=float(rho_d),
                       eps_p=float(out.eps_p) if out else math.nan,
                       eps_d=float(out.eps_d) if out else math.nan, lam_r=lam_r,
                       alpha=alpha, rank_path=rank_path, saved=saved, trace=trace,
                       time_s=time.perf_counter() - t0)


# -------------------------------------------------------------- certificate
@dataclass
class Certificate:
    rho_p: float              # residuals of one exact PDHG step from (X, y)
    rho_d: float
    primal_infeas: float      # ||A(X)-b|| + ||max(G(X)-h, 0)|| over (1 + ||[b;h]||)
    lambda_min_X: float
    dual_infeas: float        # ||min(lambda(C - M*(y)), 0)|| / (1 + ||C||_F)
    dual_sign: float          # max(y_ineq, 0)
    obj: float
    dual_obj: float
    rel_gap: float


def certificate(prob, X: np.ndarray, y: np.ndarray, alpha: float | None = None,
                row_scaling: bool = True, ops: Operators | None = None) -> Certificate:
    """Optimality certificate of any primal-dual pair (X, y) (unscaled y).

    The PDHG fixed point equals the KKT system (Section 2.1-2.2), so the
    residuals of one exact step (r = n) from (X, y) vanish iff (X, y) is
    optimal.  The other fields are the primal/dual feasibility and gap of
    the Section 1.3 primal-dual pair.
    """
    if ops is None:
        ops = Operators(prob, row_scaling=row_scaling)
    n, m = ops.n, ops.m
    alpha = 0.95 / ops.norm() if alpha is None else alpha
    ys = np.asarray(y, dtype=np.float64) * ops.scale
    C = ops.C()
    out = pdhg_step(ops, C, X, ys, n, alpha)
    rho_p = out.eps_p / (1.0 + ops.norm_C)
    rho_d = out.eps_d / (1.0 + ops.norm_rhs)
    MX = ops.apply(X)
    pin = np.linalg.norm(MX[:m] - ops.rhs[:m]) + np.linalg.norm(np.maximum(MX[m:] - ops.rhs[m:], 0))
    pin /= 1.0 + ops.norm_rhs
    lmin = float(np.linalg.eigvalsh(0.5 * (X + X.T))[0])
    S = C - ops.adjoint(ys)
    ls = np.linalg.eigvalsh(S)
    dinf = float(np.linalg.norm(np.minimum(ls, 0.0)) / (1.0 + ops.norm_C))
    dsign = float(np.max(ys[m:], initial=0.0))
    obj = float(ops.c @ svec(X))
    dual_obj = float(ops.rhs @ ys)
    gap = abs(obj - dual_obj) / (1.0 + abs(obj) + abs(dual_obj))
    return Certificate(rho_p=float(rho_p), rho_d=float(rho_d), primal_infeas=float(pin),
                       lambda_min_X=lmin, dual_infeas=dinf, dual_sign=dsign, obj=obj,
                       dual_obj=dual_obj, rel_gap=float(gap))


# ---------------------------------------------------- brute force and bounds
def brute_force_maxcut(n: int, edges: np.ndarray, weights=None) -> float:
    """Exact maximum cut by enumeration (n <= ~20)."""
    e = np.asarray(edges).reshape(-1, 2)
    w = np.ones(len(e)) if weights is None else np.asarray(weights, dtype=np.float64)
    best = 0.0
    for mask in range(1 << (n - 1)):       # vertex n-1 fixed on one side
        side = (mask >> np.arange(n)) & 1
        cut = float(np.sum(w[side[e[:, 0]] != side[e[:, 1]]]))
        best = max(best, cut)
    return best


def brute_force_min_bisection(n: int, edges: np.ndarray) -> float:
    """Exact minimum bisection (equal halves) by enumeration, n even."""
    from itertools import combinations
    e = np.asarray(edges).reshape(-1, 2)
    best = math.inf
    for S in combinations(range(1, n), n // 2 - 1):
        side = np.zeros(n, dtype=np.int64)
        side[0] = 1
        side[list(S)] = 1
        best = min(best, float(np.sum(side[e[:, 0]] != side[e[:, 1]])))
    return best


def maxcut_bracket(prob, X: np.ndarray, y: np.ndarray):
    """Certified bracket on the max-cut SDP value p* from any (X, y):

    lower = sum(y) + n min(0, lambda_min(C - Diag(y)))  (weak duality after
    shifting y to dual feasibility), upper = <C, D^{-1/2} X D^{-1/2}> with
    D = Diag(X) (a feasible primal point).  Valid for C = -L/4, diag(X) = 1.
    """
    n = prob.n
    C = dense_sym_from_coo(n, prob.c_i, prob.c_j, prob.c_v)
    lmin = float(np.linalg.eigvalsh(C - np.diag(y))[0])
    lower = float(np.sum(y) + n * min(0.0, lmin))
    d = np.sqrt(np.maximum(np.diag(X), 1e-300))
    Xf = X / np.outer(d, d)
    upper = float(np.sum(C * Xf))
    return lower, upper


# ------------------------------------------------------ hyperplane rounding
def hyperplane_round(V: np.ndarray, lam: np.ndarray, C: np.ndarray, G: np.ndarray):
    """Goemans-Williamson random-hyperplane rounding (cited in Section 1.1)
    of X = V diag(lam) V^T: trial t takes the Gaussian vector G[t] and the
    signs x_t = sign(V diag(sqrt(lam)) G[t]) (+1 where the sum is >= 0),
    i.e. the side of the hyperplane with normal G[t] on which each row vector
    of the factor V sqrt(lam) lies.  Returns (x: trials x n, values
    <C, x_t x_t^T>).  For max-cut (C = -L/4), -value is the cut weight.
    """
    F = V * np.sqrt(np.maximum(lam, 0.0))          # n x r factor of X
    S = np.asarray(G, dtype=np.float64) @ F.T       # trials x n
    x = np.where(S >= 0.0, 1.0, -1.0)
    values = np.einsum("ti,ij,tj->t", x, C, x)
    return x, values


def gw_expected_cut(X: np.ndarray, edges: np.ndarray) -> float:
    """Expected cut weight of hyperplane rounding of a unit-diagonal X
    (Goemans and Williamson's lemma): sum over edges of arccos(X_ij) / pi."""
    e = np.asarray(edges).reshape(-1, 2)
    xij = np.clip(X[e[:, 0], e[:, 1]], -1.0, 1.0)
    return float(np.sum(np.arccos(xij)) / math.pi)
