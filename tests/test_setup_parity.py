"""CPU checks of the library boundary: the C ABI loads and exports what include/namg.h declares, argument
validation rejects malformed input before any device work, and the library's host setup reproduces the
oracle's hierarchy bit for bit (C/F splittings, P and every Galerkin operator) on every level.

Host-only setup (device = -1) runs no device code, so these tests need no GPU.
"""
import os
import re

import numpy as np
import pytest

from workloads import CSR, config_system, poisson2d, poisson3d, random_csr, tridiag1d, varcoef3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def namg():
    import paper_2112_14681_amd as m

    return m


def test_library_exports_every_declared_symbol(namg):
    header = open(os.path.join(ROOT, "include", "namg.h")).read()
    body = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = set(re.findall(r"\b(namg_[a-z0-9_]+)\s*\(", body))
    assert declared == set(namg.EXPORTED)
    for name in declared:
        assert hasattr(namg.lib(), name), name


def _compare_hierarchies(namg, oracle_lib, A, **kw):
    H = namg.Hierarchy(A, device=-1, **kw)
    G = oracle_lib.Hierarchy(A, **{k: v for k, v in kw.items() if k in ("theta", "max_levels", "max_coarse",
                                                                       "ilu_levels", "agg_levels")})
    info = H.info()
    assert info["levels"] == G.levels
    for l in range(G.levels):
        e, g = H.export_level(l), G.level(l)
        Arp, Aci, Av = e["A"]
        np.testing.assert_array_equal(Arp, g.A.rowptr)
        np.testing.assert_array_equal(Aci, g.A.colind)
        assert np.array_equal(Av, g.A.vals), f"A_{l} values differ"
        if l < G.levels - 1:
            np.testing.assert_array_equal(e["cf"], g.cf)
            Prp, Pci, Pv, nc = e["P"]
            assert nc == g.P.shape[1]
            np.testing.assert_array_equal(Prp, g.P.indptr)
            np.testing.assert_array_equal(Pci, g.P.indices)
            assert np.array_equal(Pv, g.P.data), f"P_{l} values differ"
    return info


@pytest.mark.parametrize("name,N", [("c1", None), ("c2", 20), ("c2", 33), ("c3", 18), ("c4n", 14), ("c4r", 14),
                                    ("c4rcm", 14)])
def test_setup_bit_exact_vs_oracle(namg, oracle_lib, name, N):
    A, _, _ = config_system(name, N)
    info = _compare_hierarchies(namg, oracle_lib, A)
    assert info["levels"] >= 3


@pytest.mark.parametrize("theta", [0.1, 0.25, 0.5, 0.9])
def test_setup_bit_exact_theta_sweep(namg, oracle_lib, theta):
    A, _ = varcoef3d(12, 1.0, 7, 100.0)
    _compare_hierarchies(namg, oracle_lib, A, theta=theta)


def test_setup_bit_exact_random_and_small(namg, oracle_lib):
    _compare_hierarchies(namg, oracle_lib, random_csr(200, 6, 3), max_coarse=10)
    _compare_hierarchies(namg, oracle_lib, random_csr(120, 5, 4, symmetric=True), max_coarse=5)
    _compare_hierarchies(namg, oracle_lib, tridiag1d(7), max_coarse=1, max_levels=2)
    info = _compare_hierarchies(namg, oracle_lib, poisson2d(5))  # n = 25 <= 50: one level
    assert info["levels"] == 1


@pytest.mark.parametrize("name,N,agg", [("c1", None, 1), ("c1", None, 2), ("c2", 24, 2), ("c3", 20, 2), ("c4r", 14, 2),
                                        ("c2", 20, 30)])
def test_aggressive_setup_bit_exact_vs_oracle(namg, oracle_lib, name, N, agg):
    """Aggressive (A-1) coarsening on the first agg levels: C/F, P = P_1 P_2 and every Galerkin operator
    equal the oracle's bit for bit (agg = 30: every level)."""
    A, _, _ = config_system(name, N)
    info = _compare_hierarchies(namg, oracle_lib, A, agg_levels=agg)
    std = namg.Hierarchy(A, device=-1).info()
    assert info["op_complexity"] < std["op_complexity"]


def test_setup_at_64cubed_bit_exact(namg, oracle_lib):
    """A larger instance (262 144 rows, 7 levels) spanning many SELL slices and ragged coarse sizes."""
    A = poisson3d(64)
    info = _compare_hierarchies(namg, oracle_lib, A)
    assert info["levels"] == 7


def _check_ilu_factors(namg, oracle_lib, A, ilu_levels=1, **ilu):
    """The library's smoother factors on every ILU level equal the oracle's factorization of the same
    (bit-exact) level operator: L_s, U_s = D_U^{-1} strict(U) and 1/u_ii, pattern and value."""
    O = oracle_lib
    H = namg.Hierarchy(A, device=-1, ilu_levels=ilu_levels, **ilu)
    G = O.Hierarchy(A, ilu_levels=0)
    nl = H.info()["levels"]
    top = nl - 1 if ilu_levels < 0 else min(ilu_levels, nl - 1)
    for l in range(top):
        Al = G.level(l).A
        if ilu.get("ilu_kind", namg.ILU0) == namg.ILUT:
            F = O.ilut(Al, ilu["ilut_droptol"], ilu["ilut_lfil"])
        else:
            F = CSR(Al.n, Al.rowptr, Al.colind, O.ilu0(Al))
        e = H.export_ilu(l)
        rows = np.repeat(np.arange(F.n), np.diff(F.rowptr))
        lo, up, dg = F.colind < rows, F.colind > rows, F.colind == rows
        Lrp, Lci, Lv = e["L"]
        Urp, Uci, Uv = e["U"]
        np.testing.assert_array_equal(Lrp, np.concatenate([[0], np.cumsum(np.bincount(rows[lo], minlength=F.n))]))
        np.testing.assert_array_equal(Lci, F.colind[lo])
        assert np.array_equal(Lv, F.vals[lo]), l
        np.testing.assert_array_equal(Urp, np.concatenate([[0], np.cumsum(np.bincount(rows[up], minlength=F.n))]))
        np.testing.assert_array_equal(Uci, F.colind[up])
        du = F.vals[dg]
        assert np.array_equal(Uv, F.vals[up] / du[rows[up]]), l
        assert np.array_equal(e["dinv"], 1.0 / du), l
    with pytest.raises(namg.NamgError):
        H.export_ilu(top)  # the first level without factors (or the coarsest)


@pytest.mark.parametrize("name,N", [("c1", None), ("c2", 20), ("c3", 18), ("c4r", 14), ("c4n", 12)])
@pytest.mark.parametrize("ilu", [dict(), dict(ilu_kind=1, ilut_droptol=1e-2, ilut_lfil=5),
                                 dict(ilu_kind=1, ilut_droptol=1e-3, ilut_lfil=10),
                                 dict(ilu_kind=1, ilut_droptol=0.0, ilut_lfil=2)])
def test_ilu_factors_bit_exact_vs_oracle(namg, oracle_lib, name, N, ilu):
    A, _, _ = config_system(name, N)
    _check_ilu_factors(namg, oracle_lib, A, **ilu)


def test_ilut_every_level_and_nonsymmetric(namg, oracle_lib):
    """ILUT on every level but the coarsest, on a nonsymmetric random matrix and on ragged coarse levels."""
    _check_ilu_factors(namg, oracle_lib, config_system("c2", 17)[0], ilu_levels=-1, ilu_kind=namg.ILUT,
                       ilut_droptol=1e-2, ilut_lfil=5)
    _check_ilu_factors(namg, oracle_lib, random_csr(300, 7, 9), ilu_levels=-1, ilu_kind=namg.ILUT,
                       ilut_droptol=5e-3, ilut_lfil=4)


def test_pmis_setup_validation(namg):
    """The device setup needs a device and does not combine with aggressive coarsening; an unknown
    coarsening is rejected (all before any device work)."""
    A = poisson2d(12)
    assert _err(namg, lambda: namg.Hierarchy(A, device=-1, coarsen=namg.COARSEN_PMIS)) == namg.E_INVALID
    assert _err(namg, lambda: namg.Hierarchy(A, device=-1, coarsen=2)) == namg.E_INVALID
    p = namg.setup_params()
    assert (p.coarsen, p.seed) == (namg.COARSEN_RS, 0)


def test_ilut_parameter_validation(namg):
    A = poisson2d(12)
    for bad in (dict(ilu_kind=2), dict(agg_levels=-1), dict(ilu_kind=1, ilut_lfil=-1), dict(ilu_kind=1, ilut_droptol=-1e-3),
                dict(ilu_kind=1, ilut_droptol=float("nan")), dict(ilu_kind=1, ilut_droptol=float("inf"))):
        assert _err(namg, lambda: namg.Hierarchy(A, device=-1, **bad)) == namg.E_INVALID, bad
    p = namg.setup_params()
    assert (p.ilu_kind, p.ilut_lfil, p.ilut_droptol) == (namg.ILU0, 5, 1e-2)


def test_hierarchy_info_complexities(namg):
    A = poisson3d(16)
    info = namg.Hierarchy(A, device=-1).info()
    assert info["n"][0] == A.n and info["nnz"][0] == A.nnz
    assert info["op_complexity"] == pytest.approx(sum(info["nnz"]) / A.nnz)
    assert info["device_bytes"] == 0


def _err(namg, fn):
    with pytest.raises(namg.NamgError) as e:
        fn()
    return e.value.code


def test_validation_rejects_malformed_input(namg):
    A = poisson2d(6)
    # unsorted columns
    B = CSR(A.n, A.rowptr.copy(), A.colind.copy(), A.vals.copy())
    B.colind[[0, 1]] = B.colind[[1, 0]]
    assert _err(namg, lambda: namg.Hierarchy(B, device=-1)) == namg.E_INVALID
    # column out of range
    B = CSR(A.n, A.rowptr.copy(), A.colind.copy(), A.vals.copy())
    B.colind[-1] = A.n
    assert _err(namg, lambda: namg.Hierarchy(B, device=-1)) == namg.E_INVALID
    # non-monotone row pointer
    B = CSR(A.n, A.rowptr.copy(), A.colind.copy(), A.vals.copy())
    B.rowptr[3] = B.rowptr[4] + 1
    assert _err(namg, lambda: namg.Hierarchy(B, device=-1)) == namg.E_INVALID
    # non-finite value
    B = CSR(A.n, A.rowptr.copy(), A.colind.copy(), A.vals.copy())
    B.vals[5] = np.inf
    assert _err(namg, lambda: namg.Hierarchy(B, device=-1)) == namg.E_NONFINITE
    # zero / missing diagonal
    d = A.to_dense()
    d[2, 2] = 0.0
    assert _err(namg, lambda: namg.Hierarchy(CSR.from_dense(d), device=-1)) == namg.E_ZERO_PIVOT
    # bad theta
    assert _err(namg, lambda: namg.Hierarchy(A, device=-1, theta=0.0)) == namg.E_INVALID
    assert _err(namg, lambda: namg.Hierarchy(A, device=-1, theta=1.5)) == namg.E_INVALID
    # host-only hierarchy refuses device work
    H = namg.Hierarchy(A, device=-1)
    p = namg.solve_params()
    code = namg.lib().namg_solve(H.h, 1, 1, namg.C.byref(p) if hasattr(namg, "C") else None, None, None)
    assert code == namg.E_NODEVICE
    assert "host-only" in namg.lib().namg_last_error().decode()


def test_solve_param_validation(namg):
    import ctypes as C

    H = namg.Hierarchy(poisson2d(8), device=-1)
    for bad in (dict(tol=0.0), dict(restart=0), dict(restart=1000), dict(inner_terms=0), dict(smoother=7),
                dict(tri_mode=3), dict(gmres_T=2), dict(pre_sweeps=-1), dict(t_degree=0), dict(t_degree=1000), dict(stop_rule=2),
                dict(stop_rule=-1)):
        p = namg.solve_params(**bad)
        code = namg.lib().namg_solve(H.h, 1, 1, C.byref(p), None, None)
        assert code == namg.E_INVALID, bad
    with pytest.raises(TypeError):
        namg.solve_params(stop_rules=1)
    with pytest.raises(TypeError):
        namg.server_params(solve=dict(tdegree=2))
    assert namg.solve_params().stop_rule == namg.STOP_RELRES


def test_server_parameter_validation(namg):
    """Serving parameters are checked before any device work."""
    for bad in (dict(solve=dict(tri_mode=1)), dict(max_inflight=0), dict(max_inflight=1000), dict(setup_threads=0),
                dict(precision=5), dict(solve=dict(restart=0))):
        solve = bad.pop("solve", None)
        with pytest.raises(namg.NamgError) as e:
            namg.Server(solve=solve, **bad)
        assert e.value.code == namg.E_INVALID


# ------------------------------------------------------------ non-normality diagnostics (host code)
@pytest.mark.parametrize("name,N,ilu", [("c1", 20, dict()), ("c4n", 9, dict(ilu_kind=1, ilut_droptol=1e-2, ilut_lfil=5)),
                                        ("c4r", 9, dict()), ("c3", 10, dict(ilu_kind=1, ilut_droptol=1e-3, ilut_lfil=8))])
def test_ilu_diagnostics_match_oracle_definitions(namg, oracle_lib, name, N, ilu):
    """namg_ilu_diagnostics against the dense definitions (Henrici's dep via eigenvalues, ||U_s||_2 via
    the dense 2-norm, Ruiz's iteration) on the same factors: exact quantities to 1e-10, the power
    iteration's ||U_s||_2 from below to 1e-3, and the Table 2 residuals to 1e-10."""
    from oracle.nonnormal import factor_diagnostics, jacobi_tri_residuals

    O = oracle_lib
    A, _, _ = config_system(name, N)
    H = namg.Hierarchy(A, device=-1, **ilu)
    F = O.ilut(A, ilu["ilut_droptol"], ilu["ilut_lfil"]) if ilu else CSR(A.n, A.rowptr, A.colind, O.ilu0(A))
    ref = factor_diagnostics(F)
    got = H.ilu_diagnostics(0, power_iters=2000)
    assert got["n"] == A.n and got["max_row_upper"] == ref["max_row_upper"]
    assert got["ruiz_iters"] == ref["ruiz_iters"]
    for k in ("dep_L", "dep_U", "nu", "th1_bound", "th3_bound", "delta", "th4_bound", "dep_U_ruiz"):
        assert got[k] == pytest.approx(ref[k], rel=1e-10, abs=1e-12), k
    assert ref["norm2_Us"] * (1 - 1e-3) <= got["norm2_Us"] <= ref["norm2_Us"] * (1 + 1e-12)
    b = np.random.default_rng(4).standard_normal(A.n)
    for it in (0, 1, 5):
        rl, ru = H.tri_jacobi_residuals(0, b, it)
        if it == 0:
            assert rl == 1.0  # y = 0
            continue
        erl, eru = jacobi_tri_residuals(F, b, it)
        assert rl == pytest.approx(erl, rel=1e-10) and ru == pytest.approx(eru, rel=1e-10)


@pytest.mark.parametrize("name,N,ilu", [("c1", 20, dict()), ("c4n", 7, dict(ilu_kind=1, ilut_droptol=1e-2, ilut_lfil=5)),
                                        ("c3", 7, dict(ilu_kind=1, ilut_droptol=1e-3, ilut_lfil=8))])
def test_us_powers_match_oracle(namg, oracle_lib, name, N, ilu):
    """namg_us_powers against the dense powers of the same U_s (M-matrix factors, so no entry cancels and
    the nonzero counts must agree exactly): nnz exactly, max |(U_s^p)_ij| to 1e-12, the power-iteration
    ||U_s^p||_2 from below to 1e-3, through the power at which U_s^p vanishes and two beyond it."""
    from oracle.nonnormal import split_factor, us_power_sequence

    O = oracle_lib
    A, _, _ = config_system(name, N)
    H = namg.Hierarchy(A, device=-1, **ilu)
    F = O.ilut(A, ilu["ilut_droptol"], ilu["ilut_lfil"]) if ilu else CSR(A.n, A.rowptr, A.colind, O.ilu0(A))
    _, U = split_factor(F)
    depth = np.zeros(A.n, dtype=int)  # edges of the longest chain of U_s's graph from each row
    for i in range(A.n - 1, -1, -1):
        js = i + 1 + np.nonzero(U[i, i + 1:])[0]
        depth[i] = 1 + depth[js].max() if len(js) else 0
    pmax = int(depth.max()) + 2
    ref = us_power_sequence(F, pmax)
    assert ref["nnz"][pmax - 3] > 0 and ref["nnz"][pmax - 2] == 0
    got = H.us_powers(0, pmax, power_iters=2000)
    assert np.array_equal(got["nnz"], ref["nnz"])
    np.testing.assert_allclose(got["max_abs"], ref["max_abs"], rtol=1e-12, atol=0.0)
    r2 = ref["norm2"]
    assert (got["norm2"] <= r2 * (1 + 1e-12)).all() and (got["norm2"] >= r2 * (1 - 1e-3)).all()


def test_us_powers_far_powers(namg):
    """Powers far down the sequence (entries near 1e-139 on ILUT(1e-3, 20) factors of C4 at 7^3): the
    2-norm estimate never falls below the largest entry (max |t_ij| <= ||T||_2), the last nonzero power
    (a single entry here) has 2-norm equal to that entry, and every later power is reported as zero."""
    A, _, _ = config_system("c4n", 7)
    H = namg.Hierarchy(A, device=-1, ilu_levels=1, ilu_kind=namg.ILUT, ilut_droptol=1e-3, ilut_lfil=20)
    seq = H.us_powers(0, A.n, power_iters=300)
    live = seq["nnz"] > 0
    last = int(np.nonzero(live)[0].max())
    assert live[:last + 1].all() and not live[last + 1:].any()
    assert seq["max_abs"][last] < 1e-100
    assert (seq["norm2"][live] >= seq["max_abs"][live] * (1 - 1e-12)).all()
    assert seq["nnz"][last] == 1 and seq["norm2"][last] == seq["max_abs"][last]
    assert not seq["max_abs"][last + 1:].any() and not seq["norm2"][last + 1:].any()


def test_ilu_diagnostics_validation(namg):
    A = poisson2d(12)
    H = namg.Hierarchy(A, device=-1, max_coarse=200)
    for kw in (dict(power_iters=0), dict(ruiz_max_iters=-1), dict(ruiz_tol=-1.0)):
        assert _err(namg, lambda: H.ilu_diagnostics(0, **kw)) == namg.E_INVALID
    assert _err(namg, lambda: H.ilu_diagnostics(5)) == namg.E_INVALID
    H0 = namg.Hierarchy(A, device=-1, ilu_levels=0)
    assert _err(namg, lambda: H0.ilu_diagnostics(0)) == namg.E_INVALID
    assert _err(namg, lambda: H.tri_jacobi_residuals(0, np.ones(A.n), -1)) == namg.E_INVALID
    assert _err(namg, lambda: H.us_powers(0, 0)) == namg.E_INVALID
    assert _err(namg, lambda: H.us_powers(0, 3, power_iters=0)) == namg.E_INVALID
    assert _err(namg, lambda: H0.us_powers(0, 3)) == namg.E_INVALID
    with pytest.raises(ValueError):
        H.tri_jacobi_residuals(0, np.ones(A.n + 1), 3)


def test_nonnormality_study_host_only(namg):
    """bench.py's factor study runs without a GPU (host setup and diagnostics only) and reports the
    Sections 5.3.2 to 5.3.4 quantities per ordering and fill level, each within its theorem's bound; the
    powers of U_s for ILU(0) of the 7-point stencil at 7^3 vanish one step past its longest chain, 3 (7 - 1)
    edges, and ILUT's fill only lengthens the chains."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    out = bench.nonnormality_study(namg, None, 12, 10)
    assert out["gpu"] is False
    for name in ("c4n", "c4r", "c4rcm"):
        r = out["orderings"][name]
        assert r["norm2_Us"] <= r["nu"] * (1 + 1e-12) and r["nu"] <= r["th3_bound"]
        assert 0.0 < r["jacobi5_res_L"] < 1.0 and "gmres_iters" not in r
    fills = [out["fill_sweep"][k]["nnz_upper"] for k in ("5", "10", "20", "50")]
    assert fills == sorted(fills)
    pw = out["us_powers"]
    assert pw["ilu0"]["vanishes_at_p"] == 3 * (7 - 1) + 1
    assert pw["ilut_1e-3_20"]["vanishes_at_p"] >= pw["ilu0"]["vanishes_at_p"]
    for seq in (pw["ilu0"], pw["ilut_1e-3_20"]):
        assert len(seq["nnz"]) == seq["vanishes_at_p"] - 1 and min(seq["nnz"]) > 0
        assert all(m <= n2 * (1 + 1e-3) for m, n2 in zip(seq["max_abs"], seq["norm2"]))


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and says why, before touching a GPU."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_library_rs_first_pass_hand_worked_golden(namg):
    """The library's own RS first pass (host setup) on the hand-worked splittings of
    tests/golden/rs_first_pass_hand.json: the smallest-index tie-break and the weight 2 on F dependents."""
    import json

    g = json.load(open(os.path.join(ROOT, "tests", "golden", "rs_first_pass_hand.json")))
    for case in g["cases"]:
        n = case["n"]
        d = np.zeros((n, n))
        for i, j in case["edges"]:
            d[i, j] = d[j, i] = -1.0
        np.fill_diagonal(d, np.abs(d).sum(axis=1) + 1.0)
        H = namg.Hierarchy(CSR.from_dense(d), device=-1, theta=g["theta"], max_levels=2, max_coarse=1)
        assert list(H.export_level(0)["cf"]) == case["cf"], case["name"]
