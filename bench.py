"""Benchmark: time-to-1e-4 of LR-PD-SDP on max-cut G(5000, 0.01), one MI355X.

A step is one complete solve (Algorithm 2 with the truncated projection,
plain FP64) from X0 = 0, y0 = 0 until max(rho_p, rho_d) <= 1e-4 and the
rank test passes, with the problem data already resident in HBM (the
device-side restart `proxsdp_reset` is inside the timed region; host
preprocessing and the host-to-device upload happen once in `create`, outside
it, and are reported as `setup_s`).

Prints ONE JSON line on stdout.  Progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=5000)
    ap.add_argument("--p", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=1)
    ap.add_argument("--window", type=int, default=0, help="Algorithm 2 window l (0 = library default)")
    ap.add_argument("--eig-rel", type=float, default=0.0, help="eigen accuracy factor (0 = default)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see DESIGN.md for how the sweep would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import ctypes as C

    import numpy as np
    import torch

    import instances as I
    from paper_1810_05231_amd import Solver
    from paper_1810_05231_amd._lib import check, lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n = args.n
    t0 = time.perf_counter()
    prob = I.maxcut(n, args.p, args.seed)
    log(f"instance {prob.name}: n={n} edges={prob.meta['edges']} ({time.perf_counter()-t0:.1f}s)")
    t0 = time.perf_counter()
    opts = dict(tol=args.tol)
    if args.window:
        opts["window"] = args.window
    if args.eig_rel:
        opts["eig_rel"] = args.eig_rel
    s = Solver(prob, device=dev, **opts)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"create (preprocess + upload + first eigensolve): {setup_s:.2f}s, workspace "
        f"{s.ws_bytes/2**20:.0f} MiB")

    def one_solve(profile=False):
        check(lib.proxsdp_reset(s._h), "proxsdp_reset")
        if profile:
            check(lib.proxsdp_profile_enable(s._h, 1), "profile_enable")
        info = s.solve()
        prof = None
        if profile:
            pm, pc, wm, wc = C.c_double(), C.c_int32(), C.c_double(), C.c_int32()
            check(lib.proxsdp_profile_read(s._h, C.byref(pm), C.byref(pc), C.byref(wm),
                                           C.byref(wc)), "profile_read")
            prof = (pm.value, pc.value, wm.value, wc.value)
        return info, prof

    for w in range(args.warmup):
        info, _ = one_solve()
        log(f"warmup {w}: {info['status_name']} iters={info['iters']} r={info['r']} "
            f"time={info['time_s']:.3f}s obj={info['obj']:.6f}")
    torch.cuda.synchronize()
    times, infos, profs = [], [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, prof = one_solve(profile=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        infos.append(info)
        profs.append(prof)
        log(f"step {k}: {info['status_name']} iters={info['iters']} r={info['r']} "
            f"passes={info['passes']} wall={dt:.3f}s obj={info['obj']:.8f} "
            f"rho=({info['rho_p']:.2e},{info['rho_d']:.2e}) rank path {s.rank_path()}")
    ms_per_step = 1000.0 * sum(times) / len(times)
    last = infos[-1]
    dbg = s.debug()
    _, lam_f = s.factors()
    rank_x = int(np.sum(lam_f > 1e-8 * max(lam_f.max(), 1e-300))) if lam_f.size else 0
    # roofline of the dominant kernel: the dense pass Z = W B (FP64 MFMA), bytes = 8 n^2 per launch
    pass_ms = sum(p[0] for p in profs)
    pass_cnt = sum(p[1] for p in profs)
    write_ms = sum(p[2] for p in profs)
    write_cnt = sum(p[3] for p in profs)
    pass_avg_s = pass_ms / max(pass_cnt, 1) / 1000.0
    write_avg_s = write_ms / max(write_cnt, 1) / 1000.0
    bytes_pass = 8.0 * n * n
    achieved = bytes_pass / pass_avg_s / 1e9 if pass_avg_s > 0 else 0.0
    write_gbs = bytes_pass / write_avg_s / 1e9 if write_avg_s > 0 else 0.0
    roofline = {
        "kernel": "k_block_partial_f64 (dense pass W B, FP64 MFMA)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": None,
        "bytes_per_launch": bytes_pass,
        "avg_launch_us": round(pass_avg_s * 1e6, 2),
        "launches": pass_cnt,
        "unique_entry_GBps": round(8.0 * n * (n + 1) / 2 / pass_avg_s / 1e9, 1) if pass_avg_s else 0,
        "write_kernel": {"name": "k_write_w", "achieved": round(write_gbs, 1),
                         "avg_launch_us": round(write_avg_s * 1e6, 2), "launches": write_cnt},
        "sweep_share_of_solve": round((pass_ms + write_ms) / 1000.0 / max(sum(times), 1e-9), 3),
    }
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, last["iters"], args.cpu_iters)
    out = {
        "metric": "time-to-1e-4 residual (s), max-cut G(5000,0.01), plain FP64 LR-PD-SDP",
        "value": round(sum(times) / len(times), 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Erdos-Renyi graph, unit weights)",
        "config": {
            "workload": f"maxcut_G({n},{args.p})_seed{args.seed}_fp64_lr",
            "n": n, "edges": int(prob.meta["edges"]), "tol": args.tol,
            "iters": last["iters"], "final_rank": last["r"], "passes": last["passes"],
            "obj": last["obj"], "rho_p": last["rho_p"], "rho_d": last["rho_d"],
            "setup_s": round(setup_s, 3), "rank_path": s.rank_path(), "rank_X": rank_x,
            "window": args.window or 50,
            "rr_calls": int(dbg["rr_calls"]), "rr_cholesky_calls": int(dbg["rr_cholesky_calls"]),
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    s.close()


def cpu_baseline(prob, gpu_iters, iters):
    """The FP64 oracle (full eigendecomposition per iteration) timed on the host
    for `iters` PDHG iterations of the same instance, extrapolated to the GPU's
    iteration count (time-to-1e-4, seconds)."""
    import numpy as np
    try:
        import oracle as O
    except Exception as e:  # pragma: no cover
        return {"error": str(e)}
    log(f"cpu baseline: {iters} oracle iteration(s) at n={prob.n} ...")
    t0 = time.perf_counter()
    ops = O.Operators(prob)
    alpha = 0.95 / ops.norm()
    C = ops.C()
    t_setup = time.perf_counter() - t0
    X = np.zeros((prob.n, prob.n))
    y = np.zeros(prob.m + prob.p)
    t0 = time.perf_counter()
    for _ in range(iters):
        out = O.pdhg_step(ops, C, X, y, prob.n, alpha)
        X, y = out.X, out.y
    per_it = (time.perf_counter() - t0) / iters
    cores = os.cpu_count()
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([d.get("num_threads", 0) for d in info] + [1])
    except Exception:
        pass
    log(f"cpu baseline: {per_it:.2f}s per iteration")
    return {
        "value": round(per_it * gpu_iters, 1),
        "unit": "s (extrapolated time-to-1e-4)",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{iters} full-eig PDHG iteration(s) of the same n={prob.n} instance "
                  f"({per_it:.2f} s each, setup {t_setup:.1f} s excluded), times the GPU "
                  f"iteration count {gpu_iters}",
    }


if __name__ == "__main__":
    main()
