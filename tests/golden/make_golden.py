"""Write the full-size golden files: the CPU oracle's solves at the sizes the GPU tests check.

    python tests/golden/make_golden.py c2    ->  c2_128_fp64_ilu0_t3.json        (about a minute)
    python tests/golden/make_golden.py c3    ->  c3_192_fp64_pgs_t2.json         (a few minutes)
    python tests/golden/make_golden.py c4n   ->  c4n_128_fp64_ilu0_t3_m50.json   (about a minute each)
    python tests/golden/make_golden.py c4r   ->  c4r_128_fp64_ilu0_t3_m50.json
    python tests/golden/make_golden.py c4rcm ->  c4rcm_128_fp64_ilu0_t3_m50.json

Both use the benchmark's launch configuration: RS-AMG theta = 0.25 coarsened to <= 1000 rows (a dense
direct solve on the coarsest level).
c2: the benchmark's workload. 7-point Poisson, N = 128 (2 097 152 rows), b ~ N(0, 1) seed 1, hybrid V-cycle (ILU(0) on level 0, polynomial GS elsewhere)
with 3 Neumann terms, low-sync MGS-GMRES(30) with T = I - L, tol 1e-8, FP64.
c3: -div(k grad p), cell-centred, N = 192 (7 077 888 rows), lognormal k (sigma 1, seed 2), z spacing
stretched 1:100; polynomial GS with 2 Neumann terms on every level, GMRES(30), tol 1e-8, FP64 (the
reference for both the FP64 and the FP32-preconditioned GPU solves).
c4n / c4r / c4rcm: first-order upwind convection-diffusion, N = 128, Peclet 10 (seed 3), in natural order,
a random symmetric relabelling and reverse Cuthill-McKee of that; hybrid V-cycle with ILU(0) on level 0
and 3 Neumann terms, GMRES(50), tol 1e-8, FP64 (the reference for the FP64 and FP32-preconditioned
GPU solves). The orderings of Section 5.3.3.

Calls only oracle/ (and the seeded generator). Stored: level sizes and a SHA-256 of every level's C/F
array, the iteration count, the per-iteration residual estimates, the true relative residual, the max
and 2-norm of x and 4096 entries of x at seeded random positions.
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


MAX_COARSE = 1000

CONFIGS = {
    "c2": dict(file="c2_128_fp64_ilu0_t3.json", smoother="ILU0", t=3, ilu_levels=1,
               desc={"workload": "3-D Poisson 7-point", "rhs_seed": 1, "smoother": "ILU0 hybrid", "inner_terms": 3}),
    "c3": dict(file="c3_192_fp64_pgs_t2.json", smoother="PGS", t=2, ilu_levels=0,
               desc={"workload": "3-D -div(k grad p), lognormal k sigma 1, z 1:100", "k_seed": 2,
                     "smoother": "polynomial GS", "inner_terms": 2}),
}
for _o, _d in (("c4n", "natural"), ("c4r", "random symmetric relabelling"), ("c4rcm", "RCM of the random order")):
    CONFIGS[_o] = dict(file=f"{_o}_128_fp64_ilu0_t3_m50.json", smoother="ILU0", t=3, ilu_levels=1, restart=50,
                       desc={"workload": f"3-D upwind convection-diffusion, Peclet 10, {_d}", "seed": 3,
                             "smoother": "ILU0 hybrid", "inner_terms": 3})


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "c2"
    cfg = CONFIGS[name]
    A, b, meta = config_system(name)
    t0 = time.time()
    H = oracle.Hierarchy(A, theta=0.25, max_levels=25, max_coarse=MAX_COARSE, ilu_levels=cfg["ilu_levels"])
    t1 = time.time()
    levels = []
    for l in range(H.levels):
        L = H.level(l)
        entry = {"n": L.A.n, "nnz": L.A.nnz}
        if L.cf is not None:
            entry["cf_sha256"] = hashlib.sha256(np.ascontiguousarray(L.cf, dtype=np.int8).tobytes()).hexdigest()
            entry["n_coarse"] = int(L.cf.sum())
        levels.append(entry)
    smoother = oracle.SMOOTH_ILU0 if cfg["smoother"] == "ILU0" else oracle.SMOOTH_PGS
    restart = cfg.get("restart", 30)
    r = H.solve(b, tol=1e-8, restart=restart, smoother=smoother, tri_mode=oracle.TRI_NEUMANN, t=cfg["t"],
                gmres_T=oracle.T_NEUMANN)
    t2 = time.time()
    x = r["x"]
    idx = np.sort(np.random.default_rng(2024).choice(A.n, 4096, replace=False))
    out = {
        "source": f"oracle/ (CPU FP64), written by tests/golden/make_golden.py {name}",
        "config": dict(cfg["desc"], N=meta["N"], theta=0.25, max_coarse=MAX_COARSE, restart=restart, gmres_T="I-L",
                       tol=1e-8),
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
    with open(os.path.join(HERE, cfg["file"]), "w") as f:
        json.dump(out, f)
    print(f"iters {r['iters']} relres {r['relres_true']:.3e} setup {t1 - t0:.1f}s solve {t2 - t1:.1f}s")


if __name__ == "__main__":
    main()
