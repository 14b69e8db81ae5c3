"""Write cd1024_oracle_solve.json: the CPU oracle's restarted solve of the
full-size workload (2D convection-diffusion, N = 1024, n = 1,048,576,
beta = (50, 20), b ~ N(0, 1) seed 0, d = 200, k = 4, s = 400, zeta = 8,
sketch seed 0, tol = 1e-10), Algorithm 1 with the restarts of Section 3.5.

Calls only oracle/ (and the input generators in synth/).  Stored: the cycle
count, basis columns, final relative residual and the last cycle's estimates,
and |x| with x at 16 fixed indices.  Run from the repository root:
    python tests/golden/make_cd1024_oracle_solve.py [threads]
(the thread count changes only the run time: the oracle's sums have a fixed
order).
"""

from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

SAMPLE = [0, 1, 1023, 1024, 4097, 65535, 131072, 262143, 333333, 524288, 524289, 777777, 901234, 1000000,
          1048574, 1048575]


def main() -> None:
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    oracle.set_threads(threads)
    A, f, p = synth.workload("cd1024")
    nf = float(np.linalg.norm(f))
    t0 = time.perf_counter()
    rc, x, info = oracle.sgmres_solve(A, f, d=p["d"], k=p["k"], s=p["s"], zeta=p["zeta"], seed=p["seed"],
                                      tol=p["tol"], restarts=p["restarts"])
    el = time.perf_counter() - t0
    r, nrm = oracle.residual(A, f, x)
    out = {
        "workload": "cd1024",
        "params": {k: p[k] for k in ("d", "k", "s", "zeta", "seed", "tol", "restarts")},
        "rc": int(rc),
        "cycles": int(info["cycles"]),
        "steps": int(info["steps"]),
        "d_eff_last": int(info["d_eff_last"]),
        "flags": int(info["flags"]),
        "relres": float(info["relres"]),
        "relres_check": float(nrm / nf),
        "rest_est": float(info["rest_est"]),
        "kappa_est": float(info["kappa_est"]),
        "x_norm": float(np.linalg.norm(x)),
        "x_sample_index": SAMPLE,
        "x_sample": [float(x[i]) for i in SAMPLE],
        "oracle_threads": threads,
        "oracle_seconds": round(el, 1),
    }
    with open(os.path.join(HERE, "cd1024_oracle_solve.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
