"""Serving form: a request loop with continuous batching of SDP solves.

Requests (an SDP instance and an arrival time) are admitted in arrival order
while the summed device footprint of the admitted solves (their workspace,
`proxsdp_workspace_size`) stays within a budget and a slot (stream) is free.
Every admitted solve keeps its whole state (W, factors and Ritz basis, y, the
problem data) resident in its own workspace and runs on its own HIP stream,
with its check rounds replayed from captured HIP graphs; `proxsdp_step_many`
lets every solve progress independently (a round is relaunched as soon as the
previous one has been checked), so their kernels overlap on the device and no
request waits for a slower one.  The call returns as soon as a solve stops; its
slot and memory go to waiting requests at once.

Only orchestration lives here (arrival clock, admission, bookkeeping); every
iteration runs in libproxsdp.

HIP maps streams onto a small number of hardware queues (4 unless
GPU_MAX_HW_QUEUES says otherwise); streams that share a queue run one after
the other, so a process that serves many slots should export
GPU_MAX_HW_QUEUES (e.g. 16, one queue per slot) before HIP initialises.
"""
from __future__ import annotations

import collections
import dataclasses
import time

from .solver import Solver, step_many, workspace_size

__all__ = ["Request", "Result", "Server", "percentile"]


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    prob: object            # fields of proxsdp_problem (e.g. instances.Problem)


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float
    completed: float
    status: str
    iters: int
    obj: float
    rho_p: float
    rho_d: float
    footprint: int

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def percentile(xs, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    s = sorted(xs)
    if not s:
        return float("nan")
    k = max(0, min(len(s) - 1, int(-(-q * len(s) // 100)) - 1))
    return s[k]


class Server:
    """Continuous-batching request loop on one GPU.

    budget_bytes: device memory the admitted workspaces may use together.
    max_slots: largest number of solves in flight (one HIP stream each).
    solver_options: proxsdp_options fields for every solve (e.g. precision=1).
    """

    def __init__(self, device="cuda", budget_bytes=32 << 30, max_slots=16, round_iters=100,
                 **solver_options):
        import torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.round_iters = int(round_iters)   # iterations per step_many call (upper bound)
        self.opts = dict(solver_options)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.max_slots)]
        self.peak_bytes = 0
        self.peak_slots = 0

    def footprint(self, prob) -> int:
        return workspace_size(prob, **self.opts) + 256

    def run(self, requests, clock=time.perf_counter, on_done=None):
        """Serves `requests` (arrival times relative to the call) and returns
        the results in completion order."""
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        free = list(range(self.max_slots))
        active = []     # (request, solver, stream index, admitted time, footprint)
        used = 0
        results = []
        t0 = clock()
        fp_cache = {}
        while pending or active:
            now = clock() - t0
            # admission: arrival order, footprint budget, free slot
            while pending and pending[0].arrival <= now and free:
                req = pending[0]
                fp = fp_cache.get(req.rid)
                if fp is None:
                    fp = fp_cache[req.rid] = self.footprint(req.prob)
                if fp > self.budget:
                    raise ValueError(f"request {req.rid} needs {fp} bytes, above the budget")
                if used + fp > self.budget:
                    break
                pending.popleft()
                si = free.pop()
                s = Solver(req.prob, device=self.device, stream=self.streams[si], **self.opts)
                active.append((req, s, si, clock() - t0, fp))
                used += fp
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_slots = max(self.peak_slots, len(active))
            if not active:
                if pending:
                    wait = pending[0].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            # every solve progresses on its own; return as soon as one stops so
            # that its slot and memory go to a waiting request at once
            infos = step_many([a[1] for a in active], self.round_iters, until_any_stops=True)
            still = []
            for a, info in zip(active, infos):
                req, s, si, t_adm, fp = a
                if info["status_name"] == "running":
                    still.append(a)
                    continue
                res = Result(rid=req.rid, n=int(req.prob.n), arrival=req.arrival, admitted=t_adm,
                             completed=clock() - t0, status=info["status_name"],
                             iters=info["iters"], obj=info["obj"], rho_p=info["rho_p"],
                             rho_d=info["rho_d"], footprint=fp)
                if on_done is not None:
                    on_done(res, s)
                s.close()
                free.append(si)
                used -= fp
                results.append(res)
            active = still
        return results
