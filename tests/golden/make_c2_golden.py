"""Write tests/golden/c2_128_fp64_ilu0_t3.json: the CPU oracle's solve of the 128^3 Poisson system.

The configuration is the benchmark's: 7-point Poisson, N = 128 (2 097 152 rows), b ~ N(0, 1) seed 1,
RS-AMG theta = 0.25 coarsened to <= 50 rows, hybrid V-cycle (ILU(0) on level 0, polynomial GS elsewhere)
with 3 Neumann terms, low-sync MGS-GMRES(30) with T = I - L, tol 1e-8, FP64.

Calls only oracle/ (and the seeded generator). Stored: level sizes and a SHA-256 of every level's C/F
array, the iteration count, the per-iteration residual estimates, the true relative residual, the max
and 2-norm of x and 4096 entries of x at seeded random positions. Takes about a minute.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import config_system  # noqa: E402


def main():
    A, b, meta = config_system("c2")
    t0 = time.time()
    H = oracle.Hierarchy(A, theta=0.25, max_levels=25, max_coarse=50, ilu_levels=1)
    t1 = time.time()
    levels = []
    for l in range(H.levels):
        L = H.level(l)
        entry = {"n": L.A.n, "nnz": L.A.nnz}
        if L.cf is not None:
            entry["cf_sha256"] = hashlib.sha256(np.ascontiguousarray(L.cf, dtype=np.int8).tobytes()).hexdigest()
            entry["n_coarse"] = int(L.cf.sum())
        levels.append(entry)
    r = H.solve(b, tol=1e-8, restart=30, smoother=oracle.SMOOTH_ILU0, tri_mode=oracle.TRI_NEUMANN, t=3,
                gmres_T=oracle.T_NEUMANN)
    t2 = time.time()
    x = r["x"]
    idx = np.sort(np.random.default_rng(2024).choice(A.n, 4096, replace=False))
    out = {
        "source": "oracle/ (CPU FP64), written by tests/golden/make_c2_golden.py",
        "config": {"workload": "3-D Poisson 7-point", "N": meta["N"], "rhs_seed": 1, "theta": 0.25, "max_coarse": 50,
                   "smoother": "ILU0 hybrid", "inner_terms": 3, "restart": 30, "gmres_T": "I-L", "tol": 1e-8},
        "levels": levels,
        "iters": r["iters"],
        "cycles": r["cycles"],
        "hist": [float(v) for v in r["hist"]],
        "relres_true": r["relres_true"],
        "x_max_abs": float(np.abs(x).max()),
        "x_norm2": float(np.linalg.norm(x)),
        "sample_index": [int(i) for i in idx],
        "sample_x": [float(v) for v in x[idx]],
        "oracle_seconds": {"setup": round(t1 - t0, 1), "solve": round(t2 - t1, 1)},
    }
    with open(os.path.join(HERE, "c2_128_fp64_ilu0_t3.json"), "w") as f:
        json.dump(out, f)
    print(f"iters {r['iters']} relres {r['relres_true']:.3e} setup {t1 - t0:.1f}s solve {t2 - t1:.1f}s")


if __name__ == "__main__":
    main()
