"""Benchmark: time-to-1e-4 of LR-PD-SDP on max-cut G(5000, 0.01), one MI355X.

A step is one complete solve (Algorithm 2 with the truncated projection,
plain FP64) from X0 = 0, y0 = 0 until max(rho_p, rho_d) <= 1e-4 and the
rank test passes, with the problem data already resident in HBM (the
device-side restart `proxsdp_reset` is inside the timed region; host
preprocessing and the host-to-device upload happen once in `create`, outside
it, and are reported as `setup_s`).

The timed solves record no events; one further solve records HIP events on
the library's stream around every dense pass and dense write, which give the
roofline object.  The CPU leg times the oracle and, unless the workload is
sensor localisation, certifies every GPU answer (FP64 and the precision
forms) with the oracle: one exact FP64 PDHG step from it, and for max-cut the
certified bracket on the optimal value.

`--iters K` replaces the solve by K iterations (short runs for hardware
counters); `--copy-calibration MIB` first runs a plain device copy of that
size, whose counter readings calibrate the HBM byte counters.

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
PEAK_FP64_TFLOPS = 78.6      # dense FP64 MFMA
# HBM bytes per launch of the k = 64 dense pass from rocprofv3 FETCH_SIZE and
# WRITE_SIZE, calibrated against a 256 MiB device copy (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0); see profiles/k_block_partial_f64_k_write_w_n5000_k64_hbm_counters.md.
# Must be re-measured whenever k_block_partial_f64 or its chunking changes.
PASS_K64_TRAFFIC_BYTES = {"read": 209.6e6, "write": 23.3e6}
# the same counters for the dense write (tile pairs of W+) and the MFMA-busy
# fraction (rocprofv3 MfmaUtil) of both kernels at k = 64
WRITE_TRAFFIC_BYTES = {"read": 24.1e6, "write": 200.1e6}
MFMA_UTIL = {"pass": 0.447, "write": 0.161}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    # the serving stream runs one HIP stream per in-flight solve; more hardware
    # queues than HIP's default of 4 let more of them run concurrently (set
    # before HIP initialises; measured 1.2 -> 1.6 solves/s on 32 requests)
    if "--no-serving" not in sys.argv:
        slots = 16
        if "--slots" in sys.argv:
            slots = int(sys.argv[sys.argv.index("--slots") + 1])
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(max(slots, 4), 32))
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=5000)
    ap.add_argument("--p", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=4)
    ap.add_argument("--arpack-iters", type=int, default=1,
                    help="iterations of the ARPACK-style CPU baseline (0 = skip)")
    ap.add_argument("--iters", type=int, default=0, help="run K iterations instead of a solve")
    ap.add_argument("--copy-calibration", type=int, default=0, help="MiB of a plain device copy")
    ap.add_argument("--window", type=int, default=0, help="Algorithm 2 window l (0 = library default)")
    ap.add_argument("--eig-rel", type=float, default=0.0, help="eigen accuracy factor (0 = default)")
    ap.add_argument("--r0", type=int, default=0, help="initial target rank (0 = default, 1)")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16", "implicit"], default="fp64",
                    help="storage of W for the timed steps (fp32 / bf16 = precision form, "
                         "implicit = no dense W)")
    ap.add_argument("--workload", choices=["maxcut", "equip", "snl", "mimo"], default="maxcut",
                    help="maxcut / equip: G(n, p); snl: --n sensors (2000 for the full case)")
    ap.add_argument("--progress", type=int, default=0,
                    help="solve in chunks of this many iterations with a progress line each")
    ap.add_argument("--time-limit", type=float, default=0.0, help="solver time limit (s)")
    ap.add_argument("--snl-noise", type=float, default=0.0,
                    help="snl: multiplicative distance noise (0 = exact distances, as in Section 5.2)")
    ap.add_argument("--serving", type=int, default=64,
                    help="also run this many requests of the serving stream (the stream's first "
                         "requests; 512 is the whole stream)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serving-check-every", type=int, default=0,
                    help="serving: iterations per control check (0 = library default)")
    ap.add_argument("--serving-precision", choices=["fp32", "implicit"], default="fp32",
                    help="form of the served solves")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving stream")
    ap.add_argument("--serving-sat", type=int, default=32,
                    help="serving: requests of the saturation run that sets the arrival rate "
                         "(default: all of them)")
    ap.add_argument("--slots", type=int, default=16, help="serving: solves in flight")
    ap.add_argument("--budget-gib", type=float, default=32.0, help="serving: HBM budget")
    ap.add_argument("--no-precision-form", action="store_true",
                    help="skip the FP32 precision-form solve reported beside the FP64 result")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver runs on a single device and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import ctypes as C

    import numpy as np
    import torch

    import instances as I
    from paper_1810_05231_amd import Solver
    from paper_1810_05231_amd._lib import check, lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.serving_only:
        out = {"metric": "serving p50/p99 latency (s)", **serving_bench(args, dev)}
        print(json.dumps(out), flush=True)
        return
    n = args.n
    t0 = time.perf_counter()
    if args.workload == "maxcut":
        prob = I.maxcut(n, args.p, args.seed)
    elif args.workload == "equip":
        prob = I.equipartition(n, args.p, args.seed)
    elif args.workload == "mimo":
        prob = I.mimo(n, args.seed)
    else:
        prob = I.snl(n, args.seed, noise=args.snl_noise)
    log(f"instance {prob.name}: n={prob.n} m={prob.m} p={prob.p} ({time.perf_counter()-t0:.1f}s)")
    t0 = time.perf_counter()
    opts = dict(tol=args.tol)
    if args.window:
        opts["window"] = args.window
    if args.eig_rel:
        opts["eig_rel"] = args.eig_rel
    if args.r0:
        opts["r0"] = args.r0
    if args.time_limit:
        opts["time_limit_s"] = args.time_limit
    main_opts = dict(opts)
    if args.precision != "fp64":
        main_opts["precision"] = {"fp32": 1, "bf16": 2, "implicit": 3}[args.precision]
    s = Solver(prob, device=dev, **main_opts)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"create (preprocess + upload + first eigensolve): {setup_s:.2f}s, workspace "
        f"{s.ws_bytes/2**20:.0f} MiB")

    if args.copy_calibration:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration} MiB")
        del src, dst

    def one_solve(profile=False):
        check(lib.proxsdp_reset(s._h), "proxsdp_reset")
        if profile:
            check(lib.proxsdp_profile_enable(s._h, 1), "profile_enable")
        if args.iters:
            info = s.step(args.iters)
        elif args.progress:
            info = s.step(args.progress)
            while info["status_name"] == "running":
                log(f"  ... iters={info['iters']} r={info['r']} rho=({info['rho_p']:.2e},"
                    f"{info['rho_d']:.2e}) time={info['time_s']:.1f}s")
                info = s.step(args.progress)
        else:
            info = s.solve()
        prof = None
        if profile:
            tot = np.zeros(8)
            check(lib.proxsdp_profile_totals(s._h, tot.ctypes.data_as(C.POINTER(C.c_double)), 8),
                  "profile_totals")
            prof = tot
        return info, prof

    for w in range(args.warmup):
        info, _ = one_solve()
        log(f"warmup {w}: {info['status_name']} iters={info['iters']} r={info['r']} "
            f"time={info['time_s']:.3f}s obj={info['obj']:.6f}")
    torch.cuda.synchronize()
    times, infos, profs = [], [], []
    # timed solves: no profiling events on the stream
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, _ = one_solve(profile=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        infos.append(info)
        log(f"step {k}: {info['status_name']} iters={info['iters']} r={info['r']} "
            f"passes={info['passes']} verify={info['verify_steps']} wall={dt:.3f}s "
            f"obj={info['obj']:.8f} rho=({info['rho_p']:.2e},{info['rho_d']:.2e}) "
            f"rank path {s.rank_path()}")
    ms_per_step = 1000.0 * sum(times) / len(times)
    last = infos[-1]
    # one more solve with HIP events around every dense pass and dense write
    # (on the library's stream) gives the per-kernel times of the roofline
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pinfo, prof = one_solve(profile=True)
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - t0
    profs.append(prof)
    log(f"profiled solve: {pinfo['status_name']} iters={pinfo['iters']} wall={prof_wall:.3f}s")
    dbg = s.debug()
    _, lam_f = s.factors()
    rank_x = int(np.sum(lam_f > 1e-8 * max(lam_f.max(), 1e-300))) if lam_f.size else 0
    tot = np.sum(np.array(profs), axis=0)
    pass_s, pass_cnt, pass_flops, pass_bytes = tot[0] / 1e3, int(tot[1]), tot[2], tot[3]
    write_s, write_cnt, write_flops, write_bytes = tot[4] / 1e3, int(tot[5]), tot[6], tot[7]
    # Dominant sweep kernel: the dense pass Z = W B (FP64 MFMA).  Its bound is
    # the MFMA peak when its arithmetic intensity (k/4 flop/B) is above the
    # FP64 ridge (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B, i.e. k > 39), else HBM.
    intensity = pass_flops / max(pass_bytes, 1.0)
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    gbs = pass_bytes / max(pass_s, 1e-12) / 1e9
    tfs = pass_flops / max(pass_s, 1e-12) / 1e12
    if intensity > ridge:
        roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tfs / PEAK_FP64_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)}
    roofline = dict(roof)
    roofline.update({
        "traffic": (PASS_K64_TRAFFIC_BYTES["read"] + PASS_K64_TRAFFIC_BYTES["write"]
                    if (PASS_K64_TRAFFIC_BYTES and n == 5000 and args.workload == "maxcut"
                        and args.precision == "fp64") else None),
        "traffic_note": ("HBM bytes per k=64 launch (read %.1f MB + write %.1f MB of split-K "
                         "partials, rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated) vs 204.5 MB "
                         "algorithmic read" % (PASS_K64_TRAFFIC_BYTES["read"] / 1e6,
                                               PASS_K64_TRAFFIC_BYTES["write"] / 1e6)
                         if PASS_K64_TRAFFIC_BYTES else
                         "counters not taken for the current pass kernel"),
        "mfma_util_counter": MFMA_UTIL["pass"] if n == 5000 else None,
        "kernel": "k_block_partial_f64 (dense pass W B, FP64 MFMA)",
        "launches": pass_cnt,
        "avg_launch_us": round(pass_s / max(pass_cnt, 1) * 1e6, 2),
        "flops_per_launch": round(pass_flops / max(pass_cnt, 1)),
        "bytes_per_launch": round(pass_bytes / max(pass_cnt, 1)),
        "intensity_flop_per_byte": round(intensity, 2),
        "hbm_GBps": round(gbs, 1),
        "write_kernel": {"name": "k_write_w", "launches": write_cnt,
                         "avg_launch_us": round(write_s / max(write_cnt, 1) * 1e6, 2),
                         "GBps": round(write_bytes / max(write_s, 1e-12) / 1e9, 1),
                         "TFLOPs": round(write_flops / max(write_s, 1e-12) / 1e12, 2),
                         "traffic": (WRITE_TRAFFIC_BYTES["read"] + WRITE_TRAFFIC_BYTES["write"]
                                     if (n == 5000 and args.workload == "maxcut"
                                         and args.precision == "fp64") else None),
                         "mfma_util_counter": MFMA_UTIL["write"] if n == 5000 else None},
        "sweep_share_of_solve": round((pass_s + write_s) / max(prof_wall, 1e-9), 3),
        "profiled_solve_s": round(prof_wall, 4),
    })
    if pass_cnt == 0:
        roofline["note"] = ("no dense FP64 pass runs in this form (every pass applies W through its "
                            "low-rank + sparse structure); its kernel times are in "
                            "profiles/maxcut_n5000_implicit_solve_kernel_trace.md")
    # the projection sweep (dense passes + dense writes): algorithmic bytes of
    # the stored layout, and of the unique entries n(n+1)/2 of the symmetric W
    # and W+ (what a triangle-only layout would have to move), over the summed
    # kernel time
    wb = {"fp64": 8, "fp32": 4, "bf16": 2, "implicit": 0}[args.precision]
    uniq = (pass_cnt + write_cnt) * prob.n * (prob.n + 1) / 2 * wb
    sweep_s = pass_s + write_s
    roofline["sweep"] = {
        "kernels": "dense pass W B + dense write of W+",
        "bytes": pass_bytes + write_bytes,
        "seconds": round(sweep_s, 4),
        "GBps": round((pass_bytes + write_bytes) / max(sweep_s, 1e-12) / 1e9, 1),
        "frac_hbm": round((pass_bytes + write_bytes) / max(sweep_s, 1e-12) / 1e9 / PEAK_HBM_GBS, 4),
        "unique_entry_GBps": round(uniq / max(sweep_s, 1e-12) / 1e9, 1),
    }
    serving = serving_bench(args, dev) if (args.serving and not args.no_serving and not args.iters) else None
    full_cmp = None
    if args.workload != "snl" and n <= 4000 and not args.iters:
        full_cmp = full_projection_cost(s, dev, sum(times) / len(times), last)
    answers = {}
    if not args.iters:
        answers[args.precision] = s.solution(on_device=False)
    mimo_check = None
    if args.workload == "mimo" and not args.iters:
        X_ans = answers[args.precision][0]
        xhat = np.sign(X_ans[:n, n])
        errs = int(np.sum(xhat != prob.meta["x_true"]))
        mimo_check = {"bit_errors": errs, "recovered_signal": errs == 0,
                      "signal": "sign of the last column of X against the transmitted x"}
        log(f"mimo: {errs} bit errors")
    prec = None
    if not args.no_precision_form and not args.iters and args.precision == "fp64":
        prec = {}
        for name, code in (("fp32", 1), ("bf16", 2), ("implicit", 3)):
            prec[name], answers[name] = precision_form(prob, dev, opts, sum(times) / len(times),
                                                       last, code)
    cpu = None
    check_block = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, last["iters"], args.cpu_iters)
        if args.arpack_iters > 0:
            cpu["arpack_style"] = cpu_arpack_baseline(prob, last["iters"], max(int(last["r"]), 1),
                                                      args.arpack_iters)
        if answers and args.workload != "snl":
            check_block = oracle_check(prob, args.workload, answers,
                                       {args.precision: last, **(prec or {})})
    out = {
        "metric": "time-to-1e-4 residual (s)" if not args.iters else f"time for {args.iters} iterations (s)",
        "value": round(sum(times) / len(times), 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "implicit": "f64", "fp32": "f32 W / f64 Rayleigh-Ritz",
                  "bf16": "bf16 W / f64 Rayleigh-Ritz"}[args.precision],
        "data": "synthetic (seeded; Erdos-Renyi graphs with unit weights, or random sensor networks)",
        "config": {
            "workload": ({"snl": f"sensor localisation, {n} sensors, seed {args.seed}, noise {args.snl_noise}",
                          "mimo": f"binary MIMO detection, n = {n} (X in S^{n + 1}), seed {args.seed}, "
                                  f"noise sigma 0.1"}.get(args.workload,
                                                          f"{args.workload} G({n},{args.p}) seed {args.seed}"))
                        + f", {args.precision.upper()} LR-PD-SDP to {args.tol:g}",
            "n": int(prob.n), "m": int(prob.m), "p": int(prob.p), "tol": args.tol,
            "iters": last["iters"], "final_rank": last["r"], "passes": last["passes"],
            "obj": last["obj"], "rho_p": last["rho_p"], "rho_d": last["rho_d"],
            "setup_s": round(setup_s, 3), "rank_path": s.rank_path(), "rank_X": rank_x,
            "window": args.window or 50,
            "rr_calls": int(dbg["rr_calls"]), "rr_cholesky_calls": int(dbg["rr_cholesky_calls"]),
            "rr_cholesky_reasons": {"gram": int(dbg["rr_chol_gram"]),
                                    "couplings": int(dbg["rr_chol_couplings"]),
                                    "tail_bound": int(dbg["rr_chol_tail"])},
            "verify_steps": last["verify_steps"],
            "rr_newton_steps_per_call": round(dbg["rr_newton_steps_total"] / max(dbg["rr_calls"], 1), 2),
            "rr_newton_capped_calls": int(dbg["rr_newton_capped"]),
            "rr_jacobi_sweeps_after_newton": int(dbg["rr_newton_jacobi_sweeps"]),
            "rr_phase_s": {"newton": round(dbg["rr_t_newton"], 4), "cholesky": round(dbg["rr_t_cholesky"], 4),
                           "diagonalise": round(dbg["rr_t_diag"], 4), "output": round(dbg["rr_t_out"], 4)},
        },
        "roofline": roofline,
        "precision_form": prec,
        "oracle_check": check_block,
        "mimo_detection": mimo_check,
        "full_eig_comparison": full_cmp,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    s.close()


def serving_bench(args, dev):
    """Serving stream (precision form): a saturation run with every request
    present at time 0 gives the throughput; a Poisson stream at 0.7 of that
    rate gives the p50 / p99 latency (completion - arrival)."""
    import instances as I
    from paper_1810_05231_amd.serving import Request, Server, percentile
    N = args.serving or 512
    code = {"fp32": 1, "implicit": 3}[args.serving_precision]
    opts = dict(precision=code, tol=args.tol, graphs=1)
    if args.serving_check_every:
        opts["check_every"] = args.serving_check_every
    srv = Server(device=dev, budget_bytes=int(args.budget_gib * (1 << 30)), max_slots=args.slots,
                 **opts)
    Ns = min(N, args.serving_sat) if args.serving_sat > 0 else N
    base = I.serving_stream(N, seed=args.seed, rate=None)[:Ns]
    log(f"serving: {N} requests ({Ns} in the saturation run), n in [100, 2000], G(n, 8/n), "
        f"{args.serving_precision} form, {args.slots} slots")
    def progress(r, _s):
        if r.rid % 16 == 0:
            log(f"  done rid {r.rid} n={r.n} {r.status} iters={r.iters} latency={r.latency:.3f}s")

    t0 = time.perf_counter()
    res = srv.run([Request(rid, 0.0, p) for rid, _, p in base], on_done=progress)
    makespan = time.perf_counter() - t0
    thr = Ns / makespan
    ok = sum(r.status == "converged" for r in res)
    log(f"serving saturation: {makespan:.2f}s, {thr:.2f} solves/s, {ok}/{Ns} converged")
    rate = 0.7 * thr
    stream = I.serving_stream(N, seed=args.seed, rate=rate)
    t0 = time.perf_counter()
    res2 = srv.run([Request(rid, a, p) for rid, a, p in stream], on_done=progress)
    span = time.perf_counter() - t0
    lat = [r.latency for r in res2]
    ok2 = sum(r.status == "converged" for r in res2)
    out = {
        "workload": (f"first {N} of the 512-request stream" if N < 512 else "512 requests")
                    + ", max-cut/equipartition (fair coin), n ~ U[100, 2000], G(n, 8/n), "
                    + {"fp32": "FP32 precision form", "implicit": "implicit FP64 form"}[args.serving_precision]
                    + ", Poisson arrivals",
        "slots": args.slots, "budget_GiB": args.budget_gib,
        "check_every": args.serving_check_every or 10,
        "saturated_solves_per_s": round(thr, 3), "saturated_makespan_s": round(makespan, 3),
        "saturation_requests": Ns, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
        "arrival_rate_per_s": round(rate, 3),
        "p50_latency_s": round(percentile(lat, 50), 4), "p99_latency_s": round(percentile(lat, 99), 4),
        "mean_latency_s": round(sum(lat) / len(lat), 4),
        "solves_per_s": round(N / span, 3), "converged": ok2, "requests": N,
        "mean_iters": round(sum(r.iters for r in res2) / len(res2), 1),
        "peak_slots": srv.peak_slots, "peak_bytes": srv.peak_bytes,
    }
    log(f"serving stream: p50 {out['p50_latency_s']}s p99 {out['p99_latency_s']}s, "
        f"{out['solves_per_s']} solves/s, {ok2}/{N} converged")
    return out


def full_projection_cost(s, dev, t_lr, info):
    """PD-SDP's exact projection on the GPU (rocSOLVER dsyevd + reconstruction
    through proxsdp_project_psd with r = 0) timed on the solution's n x n
    matrix, against the low-rank form's whole iteration."""
    import torch
    from paper_1810_05231_amd import project_psd
    X, _ = s.solution(on_device=True)
    project_psd(X, 0)          # warm-up (library handles, code objects)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        project_psd(X, 0)
    torch.cuda.synchronize()
    full_ms = (time.perf_counter() - t0) / reps * 1e3
    lr_ms = t_lr / max(info["iters"], 1) * 1e3
    log(f"exact projection (rocSOLVER) {full_ms:.2f} ms vs LR iteration {lr_ms:.3f} ms")
    return {
        "full_eig_projection_ms": round(full_ms, 3),
        "lr_iteration_ms": round(lr_ms, 4),
        "ratio": round(full_ms / lr_ms, 2),
        "pd_sdp_projection_time_at_same_iters_s": round(full_ms * info["iters"] / 1e3, 2),
        "note": "exact projection alone (no other work), per PDHG iteration, times the LR "
                "iteration count; the LR figure is its whole iteration",
    }


def precision_form(prob, dev, opts, t64, info64, code):
    """One solve of another form of the same instance, timed like the FP64
    steps (after one untimed solve), with its difference from the plain FP64
    GPU answer: the precision form (W stored in FP32 or BF16, filter passes on
    FP32 / BF16 MFMA, exact FP64 Rayleigh-Ritz passes) or the implicit form (no
    dense W, FP64 throughout)."""
    import ctypes as C
    import numpy as np
    import torch
    from paper_1810_05231_amd import Solver
    from paper_1810_05231_amd._lib import check, lib
    s = Solver(prob, device=dev, precision=code, **opts)
    s.solve()   # warm-up (code objects, graphs of the library's first calls)
    check(lib.proxsdp_reset(s._h), "proxsdp_reset")
    check(lib.proxsdp_profile_enable(s._h, 1), "profile_enable")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = s.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tot = np.zeros(8)
    check(lib.proxsdp_profile_totals(s._h, tot.ctypes.data_as(C.POINTER(C.c_double)), 8),
          "profile_totals")
    name = {1: "fp32", 2: "bf16", 3: "implicit"}[code]
    log(f"form {name}: {info['status_name']} iters={info['iters']} r={info['r']} "
        f"passes={info['passes']} verify={info['verify_steps']} wall={dt:.3f}s obj={info['obj']:.8f}")
    form = ("no dense W: every pass applies W = V Lambda V^T + D + rank-one terms in FP64 "
            "(implicit low-rank + sparse operator)" if code == 3 else
            ("FP32" if code == 1 else "BF16") + " dense W (low-precision MFMA filter passes) "
            "+ exact FP64 Rayleigh-Ritz passes (implicit operator)")
    out = {
        "form": form,
        "value": round(dt, 4), "unit": "s", "status": info["status_name"],
        "iters": info["iters"], "passes": info["passes"], "final_rank": info["r"],
        "obj": info["obj"], "rho_p": info["rho_p"], "rho_d": info["rho_d"],
        "obj_rel_diff_vs_fp64": abs(info["obj"] - info64["obj"]) / abs(info64["obj"]),
        "speedup_vs_fp64": round(t64 / dt, 3),
        "lowp_pass_avg_us": round(tot[0] / max(tot[1], 1) * 1e3, 2),
        "lowp_pass_launches": int(tot[1]),
        "lowp_write_avg_us": round(tot[4] / max(tot[5], 1) * 1e3, 2),
        "lowp_write_launches": int(tot[5]),
    }
    ans = s.solution(on_device=False)
    s.close()
    return out, ans


def oracle_check(prob, workload, answers, infos):
    """The oracle's certificate of each GPU answer (one exact FP64 PDHG step
    from it, feasibility, duality gap) and, for max-cut, the certified bracket
    lower <= p* <= upper (weak duality at a dual-feasible shift of y; a
    rescaled feasible X), which bounds |obj - p*| without an oracle solve."""
    import oracle as O
    out = {}
    for name, (X, y) in answers.items():
        t0 = time.perf_counter()
        c = O.certificate(prob, X, y)
        obj = infos[name]["obj"]
        rec = {"cert_rho_p": c.rho_p, "cert_rho_d": c.rho_d, "cert_rho": max(c.rho_p, c.rho_d),
               "primal_infeas": c.primal_infeas, "dual_infeas": c.dual_infeas,
               "lambda_min_X": c.lambda_min_X, "rel_gap": c.rel_gap, "obj": obj}
        if workload == "maxcut":
            lo, up = O.maxcut_bracket(prob, X, y)
            rec.update({"bracket_lower": lo, "bracket_upper": up,
                        "bracket_rel_width": (up - lo) / abs(obj),
                        "obj_err_bound_rel": max(abs(obj - lo), abs(obj - up)) / abs(obj)})
        rec["seconds"] = round(time.perf_counter() - t0, 1)
        log(f"oracle check {name}: cert {rec['cert_rho']:.3e} gap {c.rel_gap:.2e}"
            + (f" bracket [{rec['bracket_lower']:.6f}, {rec['bracket_upper']:.6f}]"
               if workload == "maxcut" else "") + f" ({rec['seconds']} s)")
        out[name] = rec
    return out


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


def cpu_arpack_baseline(prob, gpu_iters, r, iters):
    """The paper's own CPU design beside the oracle: the same PDHG iteration
    with the truncated projection from ARPACK (scipy eigsh, the r algebraically
    largest eigenpairs, warm-started with the previous leading Ritz vector),
    timed for `iters` iterations and extrapolated to the GPU's iteration count.
    Uses the oracle's operators; not the oracle itself (ARPACK tolerance)."""
    import numpy as np
    from scipy.sparse.linalg import eigsh
    import oracle as O
    log(f"cpu baseline (ARPACK-style, r={r}): {iters} iteration(s) at n={prob.n} ...")
    ops = O.Operators(prob)
    alpha = 0.95 / ops.norm()
    C = ops.C()
    n, m = prob.n, prob.m
    X = np.zeros((n, n))
    y = np.zeros(m + prob.p)
    MX = ops.apply(X)
    v0 = None
    k = min(r, n - 1)
    t0 = time.perf_counter()
    for _ in range(iters):
        W = X - alpha * (C - ops.adjoint(y))
        vals, vecs = eigsh(W, k=k, which="LA", v0=v0, tol=1e-6)
        v0 = vecs[:, int(np.argmax(vals))]
        lp = np.maximum(vals, 0.0)
        Xn = (vecs * lp) @ vecs.T
        MXn = ops.apply(Xn)
        y_half = -y + alpha * (2.0 * MXn - MX)
        y = -O.dual_resolvent(y_half, alpha, ops.rhs[:m], ops.rhs[m:])
        X, MX = Xn, MXn
    per_it = (time.perf_counter() - t0) / iters
    log(f"cpu baseline (ARPACK-style): {per_it:.2f}s per iteration")
    return {
        "value": round(per_it * gpu_iters, 1),
        "unit": "s (extrapolated time-to-1e-4)",
        "kind": "ARPACK-style LR-PD-SDP (scipy eigsh 'LA', tol 1e-6, warm start)",
        "sample": f"the first {iters} iteration(s) from X = 0 at r = {k} ({per_it:.2f} s each), "
                  f"times the GPU iteration count {gpu_iters}",
    }


if __name__ == "__main__":
    main()
