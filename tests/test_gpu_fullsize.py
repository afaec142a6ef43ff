"""GPU parity at the benchmark's full size: 3-D Poisson 128^3 (2 097 152 rows), hybrid ILU(0)/poly-GS
V-cycle with 3 Neumann terms, low-sync GMRES(30) with T = I - L, FP64, in the launch configuration the
benchmark times (coarsened to <= 1000 rows, dense solve on the coarsest level).

The expected values were written by tests/golden/make_golden.py, which calls only the CPU oracle:
every level's size and C/F splitting (SHA-256), the iteration count, the residual estimate after every
iteration, and 4096 entries of the solution at seeded positions. The true residual of the GPU solution
is recomputed here with an FP64 SpMV on the host. FP64 bounds: the sampled iterate within 1e-12 of
max|x|, every residual estimate within 1e-12 of the initial relative residual (1, from x0 = 0; the first
estimate within 1e-12 relative); measured gaps are printed (PARITY-GAP lines), the largest value-by-value relative one too. The
estimate |g_i|/||b|| is a relative residual: summation order perturbs it by about eps ||r_0|| however small
|g_i| has become, so it is compared in the same max-norm sense as the iterate.
Also at full size: C3 (192^3) and the three orderings of C4 (128^3, GMRES(50)).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle as O
from workloads import config_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_128_fp64_ilu0_t3.json")
SOLVE = dict(smoother=1, tri_mode=0, inner_terms=3, restart=30, gmres_T=0, tol=1e-8)
MAX_COARSE = 1000  # the benchmark's coarsest-level bound for C2 and C3


@pytest.fixture(scope="module")
def namg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_14681_amd as m

    return m


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def system(namg):
    A, b, meta = config_system("c2")
    assert meta["N"] == 128
    H = namg.Hierarchy(A, device=0, ilu_levels=1, max_coarse=MAX_COARSE)
    return A, b, H


def _solve(namg, H, b, **kw):
    bt = torch.from_numpy(b).to("cuda:0")
    xt = torch.zeros_like(bt)
    st = H.solve(bt, xt, **dict(SOLVE, **kw))
    torch.cuda.synchronize()
    return st, xt.cpu().numpy()


def test_hierarchy_matches_oracle(namg, golden, system):
    A, b, H = system
    info = H.info()
    assert info["levels"] == len(golden["levels"])
    for l, g in enumerate(golden["levels"]):
        assert (info["n"][l], info["nnz"][l]) == (g["n"], g["nnz"]), l
        if "cf_sha256" in g:
            cf = np.ascontiguousarray(H.export_level(l)["cf"], dtype=np.int8)
            assert hashlib.sha256(cf.tobytes()).hexdigest() == g["cf_sha256"], l
            assert int(cf.sum()) == g["n_coarse"]


def _check_fp64_against_golden(namg, label, A, b, st, x, golden):
    """Iterations, every residual estimate, the sampled iterate, ||x|| and the true residual."""
    idx = np.asarray(golden["sample_index"])
    xmax = golden["x_max_abs"]
    gx = float(np.abs(x[idx] - np.asarray(golden["sample_x"])).max() / xmax)
    h, gh_ref = np.asarray(st["hist"]), np.asarray(golden["hist"])
    assert h.shape == gh_ref.shape, (h.shape, gh_ref.shape)
    d = np.abs(h - gh_ref)
    gh = float(d.max())  # the estimates are relative to ||b||, and x0 = 0: the initial one is 1
    gh0 = float(d[0] / abs(gh_ref[0]))
    ghv = float((d / np.abs(gh_ref)).max())
    gn = abs(np.linalg.norm(x) - golden["x_norm2"]) / golden["x_norm2"]
    res = np.linalg.norm(b - O.spmv(A, x)) / np.linalg.norm(b)
    print(f"PARITY-GAP {label} iters={st['iters']} (oracle {golden['iters']}) x_sample={gx:.2e} hist={gh:.2e} "
          f"hist_first={gh0:.2e} hist_value_by_value={ghv:.2e} norm={gn:.2e} relres={res:.3e}")
    assert st["status"] == namg.OK
    assert st["iters"] == golden["iters"] and st["cycles"] == golden["cycles"]
    assert gh <= 1e-12, gh
    assert gh0 <= 1e-12, gh0
    assert gx <= 1e-12, gx
    assert gn <= 1e-12, gn
    assert np.abs(x).max() == pytest.approx(xmax, rel=1e-12)
    assert res <= 1e-8
    assert st["relres_true"] == pytest.approx(res, rel=1e-6)
    assert st["relres_true"] == pytest.approx(golden["relres_true"], rel=1e-6)


def test_full_solve_matches_oracle(namg, golden, system):
    A, b, H = system
    st, x = _solve(namg, H, b, history=True)
    _check_fp64_against_golden(namg, "c2 128^3 fp64", A, b, st, x, golden)


def test_stop_after_k_iterations(namg, golden, system):
    """Stopping after k < the converged count reports NOT_CONVERGED with the oracle's k-th estimate."""
    A, b, H = system
    for k in (1, golden["iters"] // 2, golden["iters"] - 1):
        st, _ = _solve(namg, H, b, max_iters=k)
        assert st["status"] == namg.NOT_CONVERGED and st["iters"] == k
        assert abs(st["relres_est"] - golden["hist"][k - 1]) <= 1e-12, k


def test_fp32_preconditioner_full_size(namg, golden, system):
    A, b, _ = system
    H32 = namg.Hierarchy(A, device=0, precision=namg.FP32_PRECOND, ilu_levels=1, max_coarse=MAX_COARSE)
    st, x = _solve(namg, H32, b)
    res = np.linalg.norm(b - O.spmv(A, x)) / np.linalg.norm(b)
    assert st["status"] == namg.OK and res <= 1e-8
    assert abs(st["iters"] - golden["iters"]) <= 2
    idx = np.asarray(golden["sample_index"])
    assert np.abs(x[idx] - np.asarray(golden["sample_x"])).max() / golden["x_max_abs"] <= 1e-6


# ------------------------------------------------------------------------------------ C3 at 192^3
GOLDEN_C3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_192_fp64_pgs_t2.json")
SOLVE_C3 = dict(smoother=0, tri_mode=0, inner_terms=2, restart=30, gmres_T=0, tol=1e-8)


@pytest.fixture(scope="module")
def golden_c3():
    with open(GOLDEN_C3) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def system_c3(namg):
    A, b, meta = config_system("c3")
    assert meta["N"] == 192
    return A, b


def test_c3_fp64_matches_oracle(namg, golden_c3, system_c3):
    """-div(k grad p) at 192^3 (7 077 888 rows, lognormal k, z stretched 1:100), polynomial GS t = 2."""
    A, b = system_c3
    H = namg.Hierarchy(A, device=0, ilu_levels=0, max_coarse=MAX_COARSE)
    info = H.info()
    assert info["levels"] == len(golden_c3["levels"])
    for l, g in enumerate(golden_c3["levels"]):
        assert (info["n"][l], info["nnz"][l]) == (g["n"], g["nnz"]), l
    cf0 = np.ascontiguousarray(H.export_level(0)["cf"], dtype=np.int8)
    assert hashlib.sha256(cf0.tobytes()).hexdigest() == golden_c3["levels"][0]["cf_sha256"]
    st, x = _solve(namg, H, b, history=True, **SOLVE_C3)
    H.close()
    _check_fp64_against_golden(namg, "c3 192^3 fp64", A, b, st, x, golden_c3)


def test_c3_fp32_preconditioner(namg, golden_c3, system_c3):
    """The C3 configuration's FP32 hierarchy and V-cycle under FP64 GMRES: the same 1e-8 true residual
    (independent FP64 SpMV) in at most two more iterations than the FP64 oracle."""
    A, b = system_c3
    H = namg.Hierarchy(A, device=0, precision=namg.FP32_PRECOND, ilu_levels=0, max_coarse=MAX_COARSE)
    st, x = _solve(namg, H, b, **SOLVE_C3)
    H.close()
    res = np.linalg.norm(b - O.spmv(A, x)) / np.linalg.norm(b)
    assert st["status"] == namg.OK and res <= 1e-8
    assert abs(st["iters"] - golden_c3["iters"]) <= 2
    idx = np.asarray(golden_c3["sample_index"])
    gap = np.abs(x[idx] - np.asarray(golden_c3["sample_x"])).max() / golden_c3["x_max_abs"]
    print(f"C3 FP32: iters {st['iters']}, relres {res:.2e}, sampled |x - x_oracle| / max|x| = {gap:.2e}")
    # measured 1.4e-13: the residual left at 1e-8 lies in the stiff (large-eigenvalue) components, which
    # carry little of x; the bound keeps five orders of margin
    assert gap <= 1e-8, gap


# ------------------------------------------------------------------------------ C4 orderings at 128^3
SOLVE_C4 = dict(smoother=1, tri_mode=0, inner_terms=3, restart=50, gmres_T=0, tol=1e-8)


@pytest.mark.parametrize("name", ["c4n", "c4r", "c4rcm"])
def test_c4_orderings_full_size(namg, name):
    """Upwind convection-diffusion at 128^3 in natural, random and RCM order (Section 5.3.3), hybrid ILU(0)
    t = 3, GMRES(50): every level's size and C/F splitting equal the oracle's, the FP64 solve matches the
    oracle (iterations, every residual estimate, sampled iterate), and the FP32 preconditioner reaches the
    same 1e-8 true residual."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_128_fp64_ilu0_t3_m50.json")
    with open(path) as f:
        g = json.load(f)
    A, b, meta = config_system(name)
    assert meta["N"] == 128
    H = namg.Hierarchy(A, device=0, ilu_levels=1, max_coarse=MAX_COARSE)
    info = H.info()
    assert info["levels"] == len(g["levels"])
    for l, gl in enumerate(g["levels"]):
        assert (info["n"][l], info["nnz"][l]) == (gl["n"], gl["nnz"]), l
        if "cf_sha256" in gl:
            cf = np.ascontiguousarray(H.export_level(l)["cf"], dtype=np.int8)
            assert hashlib.sha256(cf.tobytes()).hexdigest() == gl["cf_sha256"], l
    st, x = _solve(namg, H, b, history=True, **SOLVE_C4)
    H.close()
    _check_fp64_against_golden(namg, f"{name} 128^3 fp64", A, b, st, x, g)
    H32 = namg.Hierarchy(A, device=0, precision=namg.FP32_PRECOND, ilu_levels=1, max_coarse=MAX_COARSE)
    st, x = _solve(namg, H32, b, **SOLVE_C4)
    H32.close()
    res = np.linalg.norm(b - O.spmv(A, x)) / np.linalg.norm(b)
    idx = np.asarray(g["sample_index"])
    gap = np.abs(x[idx] - np.asarray(g["sample_x"])).max() / g["x_max_abs"]
    print(f"PARITY-GAP {name} 128^3 fp32 iters={st['iters']} (oracle {g['iters']}) relres={res:.3e} x_sample={gap:.2e}")
    assert st["status"] == namg.OK and res <= 1e-8
    assert abs(st["iters"] - g["iters"]) <= 2
    assert gap <= 1e-6, gap
