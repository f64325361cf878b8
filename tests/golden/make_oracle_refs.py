"""Writes oracle_refs.json: the FP64 oracle's answers (objective, iterations,
final rank, certificate) on the seeded test instances whose oracle solves take
too long to repeat inside a GPU test.  Calls only ``oracle`` and ``instances``.

    python tests/golden/make_oracle_refs.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import instances as I  # noqa: E402
import oracle as O  # noqa: E402

# (kind, n, edge probability, seed, tol)
CASES = [
    ("maxcut", 400, 0.05, 5, 1e-4),
    ("equip", 300, 0.05, 6, 1e-4),
]


def key(kind, n, p, seed, tol):
    return f"{kind}_n{n}_p{p}_s{seed}_tol{tol:g}"


def main():
    out = {}
    for kind, n, p, seed, tol in CASES:
        prob = I.maxcut(n, p, seed) if kind == "maxcut" else I.equipartition(n, p, seed)
        t0 = time.perf_counter()
        res = O.solve(prob, tol=tol, max_iters=200000)
        cert = O.certificate(prob, res.X, res.y)
        out[key(kind, n, p, seed, tol)] = {
            "status": O.STATUS_NAMES[res.status], "iters": res.iters, "r": res.r,
            "obj": res.obj, "dual_obj": res.dual_obj, "rho_p": res.rho_p, "rho_d": res.rho_d,
            "cert_rho": max(cert.rho_p, cert.rho_d), "cert_rel_gap": cert.rel_gap,
            "seconds": round(time.perf_counter() - t0, 1),
        }
        print(key(kind, n, p, seed, tol), out[key(kind, n, p, seed, tol)], flush=True)
    with open(os.path.join(HERE, "oracle_refs.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
