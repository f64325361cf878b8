"""Python-facing wrappers of libproxsdp (argument marshalling only).

PyTorch supplies device memory (the workspace tensors) and the stream; every
step of the method runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import FP64, Info, Problem, check, default_options, lib

__all__ = ["Solver", "project_psd", "project_psd_noalloc", "problem_struct", "workspace_size",
           "step_many"]


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a.size else None


def problem_struct(prob):
    """ctypes Problem view of an object with the fields of the C struct.

    Returns (struct, keepalive) -- keep the second item alive while the
    struct is in use.
    """
    arrs = dict(
        c_i=np.ascontiguousarray(prob.c_i, dtype=np.int32),
        c_j=np.ascontiguousarray(prob.c_j, dtype=np.int32),
        c_v=np.ascontiguousarray(prob.c_v, dtype=np.float64),
        a_row=np.ascontiguousarray(prob.a_row, dtype=np.int32),
        a_i=np.ascontiguousarray(prob.a_i, dtype=np.int32),
        a_j=np.ascontiguousarray(prob.a_j, dtype=np.int32),
        a_v=np.ascontiguousarray(prob.a_v, dtype=np.float64),
        r1_row=np.ascontiguousarray(getattr(prob, "r1_row", np.zeros(0)), dtype=np.int32),
        r1_sigma=np.ascontiguousarray(getattr(prob, "r1_sigma", np.zeros(0)), dtype=np.float64),
        r1_u=np.ascontiguousarray(getattr(prob, "r1_u", np.zeros(0)), dtype=np.float64).reshape(-1),
        b=np.ascontiguousarray(prob.b, dtype=np.float64),
        h=np.ascontiguousarray(prob.h, dtype=np.float64),
    )
    s = Problem()
    s.n, s.m, s.p = int(prob.n), int(prob.m), int(prob.p)
    s.nnz_c = arrs["c_v"].size
    s.c_i, s.c_j, s.c_v = (_ptr(arrs["c_i"], C.c_int32), _ptr(arrs["c_j"], C.c_int32),
                           _ptr(arrs["c_v"], C.c_double))
    s.nnz_a = arrs["a_v"].size
    s.a_row, s.a_i, s.a_j = (_ptr(arrs["a_row"], C.c_int32), _ptr(arrs["a_i"], C.c_int32),
                             _ptr(arrs["a_j"], C.c_int32))
    s.a_v = _ptr(arrs["a_v"], C.c_double)
    s.n_r1 = arrs["r1_row"].size
    s.r1_row = _ptr(arrs["r1_row"], C.c_int32)
    s.r1_sigma = _ptr(arrs["r1_sigma"], C.c_double)
    s.r1_u = _ptr(arrs["r1_u"], C.c_double)
    s.b = _ptr(arrs["b"], C.c_double)
    s.h = _ptr(arrs["h"], C.c_double)
    return s, arrs


def workspace_size(prob, **options) -> int:
    s, keep = problem_struct(prob)
    o = default_options(**options)
    nb = C.c_size_t()
    check(lib.proxsdp_workspace_size(C.byref(s), C.byref(o), C.byref(nb)),
          "proxsdp_workspace_size")
    return int(nb.value)


def _device_buffer(nbytes: int, device):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    addr = buf.data_ptr()
    off = (-addr) % 256
    return buf, addr + off


def _stream_handle(device):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver:
    """LR-PD-SDP / PD-SDP solver on one GPU.

    ``prob`` is any object with the fields of ``proxsdp_problem`` as numpy
    arrays (``instances.Problem`` is one).  Options are the fields of
    ``proxsdp_options``.
    """

    def __init__(self, prob, device="cuda", stream=None, **options):
        """`stream`: a torch.cuda.Stream the handle runs on (default: the
        current stream); the workspace is allocated on it."""
        import torch
        self.device = torch.device(device)
        self.n = int(prob.n)
        self.rows = int(prob.m) + int(prob.p)
        s, keep = problem_struct(prob)
        o = default_options(**options)
        nb = C.c_size_t()
        check(lib.proxsdp_workspace_size(C.byref(s), C.byref(o), C.byref(nb)),
              "proxsdp_workspace_size")
        self.ws_bytes = int(nb.value)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(self.stream):
            self._buf, ptr = _device_buffer(self.ws_bytes, self.device)
        self._h = C.c_void_p()
        check(lib.proxsdp_create(C.byref(s), C.byref(o), C.c_void_p(ptr), self.ws_bytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(self._h)),
              "proxsdp_create")
        del keep

    def step(self, n_iters: int = 1) -> dict:
        info = Info()
        check(lib.proxsdp_step(self._h, int(n_iters), C.byref(info)), "proxsdp_step")
        return info.to_dict()

    def solve(self) -> dict:
        info = Info()
        check(lib.proxsdp_solve(self._h, C.byref(info)), "proxsdp_solve")
        return info.to_dict()

    def solution(self, on_device: bool = True):
        """(X, y): X as an n x n float64 tensor (device) or ndarray, y as ndarray.

        X is always formed on the device (dense write from the factors) and
        copied to the host when on_device is False."""
        import torch
        y = np.zeros(self.rows)
        X = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        check(lib.proxsdp_get_solution(self._h, None, y.ctypes.data_as(C.c_void_p), 0),
              "get_solution(y)")
        check(lib.proxsdp_get_solution(self._h, C.c_void_p(X.data_ptr()), None, 1),
              "get_solution(X)")
        torch.cuda.synchronize(self.device)
        return (X, y) if on_device else (X.cpu().numpy(), y)

    def factors(self):
        r = C.c_int32()
        check(lib.proxsdp_get_factors(self._h, None, None, C.byref(r)), "get_factors")
        V = np.zeros((self.n, max(r.value, 1)))
        lam = np.zeros(max(r.value, 1))
        check(lib.proxsdp_get_factors(self._h, V.ctypes.data_as(C.POINTER(C.c_double)),
                                      lam.ctypes.data_as(C.POINTER(C.c_double)), C.byref(r)),
              "get_factors")
        return V[:, :r.value], lam[:r.value]

    def get_state(self):
        """(V, lambda, y) of the current iterate (X = V diag(lambda) V^T, y unscaled)."""
        r = C.c_int32()
        check(lib.proxsdp_get_state(self._h, None, None, None, C.byref(r)), "get_state")
        V = np.zeros((self.n, max(r.value, 1)))
        lam = np.zeros(max(r.value, 1))
        y = np.zeros(self.rows)
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        check(lib.proxsdp_get_state(self._h, p(V), p(lam), p(y), C.byref(r)), "get_state")
        return V[:, :r.value].copy(), lam[:r.value].copy(), y

    def set_state(self, V, lam, y=None) -> None:
        """Warm start from X0 = V diag(lam) V^T and y0 (unscaled; None = 0)."""
        V = np.ascontiguousarray(V, dtype=np.float64).reshape(self.n, -1)
        lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
        r = lam.size
        if V.shape[1] != r:
            raise ValueError("V must have one column per lambda")
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        yy = None if y is None else np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
        if yy is not None and yy.size != self.rows:
            raise ValueError(f"y must have {self.rows} values")
        check(lib.proxsdp_set_state(self._h, r, p(V) if r else None, p(lam) if r else None,
                                    p(yy) if yy is not None else None), "set_state")

    def reset(self) -> None:
        """Restart from X0 = 0, y0 = 0 on the data already on the device."""
        check(lib.proxsdp_reset(self._h), "proxsdp_reset")

    def rank_path(self):
        """[(iteration, new r, reason)] with reason 1 = rank test failed at
        convergence, 2 = windowed residual test found no decrease."""
        cnt = C.c_int32()
        check(lib.proxsdp_rank_path(self._h, None, None, None, 0, C.byref(cnt)), "rank_path")
        m = max(cnt.value, 1)
        it = np.zeros(m, np.int32)
        rk = np.zeros(m, np.int32)
        why = np.zeros(m, np.int32)
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        check(lib.proxsdp_rank_path(self._h, p(it), p(rk), p(why), m, C.byref(cnt)), "rank_path")
        return [(int(a), int(b), int(c)) for a, b, c in zip(it, rk, why)][:cnt.value]

    def debug(self) -> dict:
        """Internal device scalars (see proxsdp_debug_scalars)."""
        out = np.zeros(64 + 64)
        check(lib.proxsdp_debug_scalars(self._h, out.ctypes.data_as(C.POINTER(C.c_double)),
                                        out.size), "debug_scalars")
        names = {0: "alpha", 1: "lower_bound", 2: "maxres", 3: "lambda_r", 4: "lambda_r1",
                 5: "normw", 6: "eps_p", 7: "eps_d", 8: "obj", 9: "dual_obj", 10: "dx2",
                 13: "nonfinite", 14: "dropped", 15: "filter_c", 16: "filter_e", 17: "sweeps",
                 18: "rr_newton_steps", 19: "rr_cholesky_calls", 20: "rr_calls",
                 22: "rr_chol_gram", 23: "rr_chol_couplings", 24: "rr_chol_tail",
                 25: "rr_t_newton", 26: "rr_t_cholesky", 27: "rr_t_diag", 28: "rr_t_out",
                 29: "npos", 30: "filter_x1", 31: "rr_newton_steps_total",
                 32: "rr_newton_capped", 33: "rr_newton_jacobi_sweeps"}
        d = {v: float(out[k]) for k, v in names.items()}
        d["theta"] = out[64:].tolist()
        return d

    def saved(self):
        """Algorithm 2's intermediate feasible solutions X_[r] kept so far:
        [(iteration, V, lambda, y)] with X_[r] = V diag(lambda) V^T, y unscaled."""
        cnt = C.c_int32()
        check(lib.proxsdp_saved_count(self._h, C.byref(cnt)), "saved_count")
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        out = []
        for i in range(cnt.value):
            r = C.c_int32()
            it = C.c_int32()
            check(lib.proxsdp_get_saved(self._h, i, None, None, None, C.byref(r), C.byref(it)),
                  "get_saved")
            V = np.zeros((self.n, max(r.value, 1)))
            lam = np.zeros(max(r.value, 1))
            y = np.zeros(self.rows)
            check(lib.proxsdp_get_saved(self._h, i, p(V), p(lam), p(y), C.byref(r), C.byref(it)),
                  "get_saved")
            out.append((int(it.value), V[:, :r.value].copy(), lam[:r.value].copy(), y))
        return out

    def round_hyperplane(self, g):
        """Random-hyperplane rounding of the current iterate with the Gaussian
        vectors g (trials x r, r = the current rank).  Returns (values
        <C, x x^T> per trial, x of the best trial as int8 +-1, its index)."""
        g = np.ascontiguousarray(g, dtype=np.float64)
        trials = g.shape[0]
        values = np.zeros(trials)
        x = np.zeros(self.n, dtype=np.int8)
        best = C.c_int32()
        check(lib.proxsdp_round_hyperplane(
            self._h, trials, g.ctypes.data_as(C.POINTER(C.c_double)) if g.size else None,
            values.ctypes.data_as(C.POINTER(C.c_double)), x.ctypes.data_as(C.POINTER(C.c_int8)),
            C.byref(best)), "round_hyperplane")
        return values, x, int(best.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.proxsdp_destroy(self._h)
            self._h = C.c_void_p()
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STEP_UNTIL_ANY_STOPS = 1


def step_many(solvers, n_iters: int, until_any_stops: bool = False):
    """Advances several solvers (each on its own stream) by up to n_iters
    iterations, each progressing independently on the device; with
    until_any_stops the call returns once one of them stops.  Returns their
    info dicts."""
    cnt = len(solvers)
    if cnt == 0:
        return []
    hs = (C.c_void_p * cnt)(*[s._h.value for s in solvers])
    infos = (Info * cnt)()
    check(lib.proxsdp_step_many(hs, cnt, int(n_iters),
                                STEP_UNTIL_ANY_STOPS if until_any_stops else 0,
                                C.cast(infos, C.c_void_p)), "proxsdp_step_many")
    return [infos[i].to_dict() for i in range(cnt)]


def project_psd(S, r: int, tol: float = 1e-12, want_P: bool = True, want_vectors: bool = False):
    """aproj(S, r) for a device float64 tensor S (n x n, row stride S.stride(0)).

    Returns (P or None, eigenvalues (r, decreasing), eigenvectors (n x r) or
    None, number of positive kept eigenvalues).
    """
    import torch
    assert S.is_cuda and S.dtype == torch.float64 and S.dim() == 2 and S.stride(1) == 1
    n = S.shape[0]
    re = n if (r <= 0 or r >= n) else r
    nb = C.c_size_t()
    check(lib.proxsdp_project_workspace_size(n, int(r), FP64, C.byref(nb)),
          "proxsdp_project_workspace_size")
    buf, ptr = _device_buffer(int(nb.value), S.device)
    P = torch.empty((n, n), dtype=torch.float64, device=S.device) if want_P else None
    evals = np.zeros(re)
    evecs = np.zeros((n, re)) if want_vectors else None
    rank = C.c_int32()
    check(lib.proxsdp_project_psd(
        C.c_void_p(S.data_ptr()), n, S.stride(0), int(r), FP64, float(tol),
        C.c_void_p(P.data_ptr()) if P is not None else None, n,
        evals.ctypes.data_as(C.POINTER(C.c_double)),
        evecs.ctypes.data_as(C.POINTER(C.c_double)) if evecs is not None else None,
        C.byref(rank), C.c_void_p(ptr), int(nb.value), _stream_handle(S.device)),
        "proxsdp_project_psd")
    del buf
    return P, evals, evecs, int(rank.value)


def project_psd_noalloc(S, r: int, tol: float = 1e-12, P=None, want_vectors: bool = False):
    """proxsdp_project_psd_noalloc: aproj(S, r) with the library's static
    device scratch instead of a workspace.  ``P``: a preallocated n x n float64
    device tensor (or None).  Returns (P, eigenvalues, eigenvectors or None,
    number of positive kept eigenvalues)."""
    import torch
    assert S.is_cuda and S.dtype == torch.float64 and S.dim() == 2 and S.stride(1) == 1
    n = S.shape[0]
    re = n if (r <= 0 or r >= n) else r
    if P is not None:
        assert P.is_cuda and P.dtype == torch.float64 and P.stride(1) == 1 and P.shape[0] >= n
    evals = np.zeros(re)
    evecs = np.zeros((n, re)) if want_vectors else None
    rank = C.c_int32()
    check(lib.proxsdp_project_psd_noalloc(
        C.c_void_p(S.data_ptr()), n, S.stride(0), int(r), FP64, float(tol),
        C.c_void_p(P.data_ptr()) if P is not None else None, P.stride(0) if P is not None else n,
        evals.ctypes.data_as(C.POINTER(C.c_double)),
        evecs.ctypes.data_as(C.POINTER(C.c_double)) if evecs is not None else None,
        C.byref(rank), _stream_handle(S.device)), "proxsdp_project_psd_noalloc")
    return P, evals, evecs, int(rank.value)
