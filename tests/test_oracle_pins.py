"""Pins of the CPU oracle against facts fixed by the paper and by mathematics, not by the oracle itself.

Each test names the passage or the closed form that fixes the expected value. Independent routes are
numpy/scipy dense linear algebra, closed-form Poisson eigenpairs, brute-force structure checks and the
golden fixtures under tests/golden/.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from workloads import CSR, poisson2d, poisson3d, random_csr, tridiag1d, varcoef3d, convdiff3d

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------------------------- SpMV
def test_spmv_matches_dense_product(oracle_lib):
    O = oracle_lib
    for seed in range(3):
        A = random_csr(40, 6, seed)
        x = np.random.default_rng(seed).standard_normal(A.n)
        np.testing.assert_allclose(O.spmv(A, x), A.to_dense() @ x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("N", [5, 9])
def test_spmv_poisson_eigenvectors_2d_3d(oracle_lib, N):
    """A v = lambda v for v_jk = sin(j pi x/(N+1)) sin(k pi y/(N+1)), lambda = 4 - 2cos - 2cos (3-D: 6 - sum)."""
    O = oracle_lib
    g = np.arange(1, N + 1) / (N + 1)
    A2 = poisson2d(N)
    for (j, k) in [(1, 1), (2, 3), (N, 1)]:
        v = np.outer(np.sin(k * np.pi * g), np.sin(j * np.pi * g)).ravel()  # x fastest
        lam = 4 - 2 * np.cos(j * np.pi / (N + 1)) - 2 * np.cos(k * np.pi / (N + 1))
        np.testing.assert_allclose(O.spmv(A2, v), lam * v, atol=1e-13)
    A3 = poisson3d(N)
    for (i, j, k) in [(1, 1, 1), (2, 1, 3)]:
        v = np.einsum("a,b,c->abc", np.sin(k * np.pi * g), np.sin(j * np.pi * g), np.sin(i * np.pi * g)).ravel()
        lam = 6 - 2 * sum(np.cos(q * np.pi / (N + 1)) for q in (i, j, k))
        np.testing.assert_allclose(O.spmv(A3, v), lam * v, atol=1e-13)


# ------------------------------------------------------------------------------------ strength / RS
def test_strength_threshold_hand_example(oracle_lib):
    """Section 5.1: j strongly influences i iff |a_ij| >= theta max_{k != i} |a_ik| (theta = 0.25)."""
    d = np.array([[4.0, -1.0, -0.25, 0.0], [-0.2, 3.0, -1.0, -0.1], [0.0, -0.5, 2.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
    srp, sci = oracle_lib.strength(CSR.from_dense(d), 0.25)
    rows = [list(sci[srp[i]:srp[i + 1]]) for i in range(4)]
    # row 0: max 1 -> thr 0.25: both -1 and -0.25 qualify (ties count); row 1: max 1 -> thr .25: only col 2
    # row 2: only neighbour col 1; row 3: no off-diagonal -> empty
    assert rows == [[1, 2], [2], [1], []]


def test_rs_tridiag_golden(oracle_lib):
    g = json.load(open(os.path.join(GOLD, "tridiag7_rs.json")))
    A = tridiag1d(7)
    assert list(oracle_lib.coarsen(A, g["theta"])) == g["cf"]
    H = oracle_lib.Hierarchy(A, theta=g["theta"], max_levels=2, max_coarse=1)
    L0 = H.level(0)
    np.testing.assert_array_equal(L0.cf, g["cf"])
    np.testing.assert_array_equal(L0.P.toarray(), np.array(g["P"]))
    np.testing.assert_array_equal(H.level(1).A.to_dense(), np.array(g["Ac"]))


def _strong_sets(O, A, theta):
    srp, sci = O.strength(A, theta)
    return [set(sci[srp[i]:srp[i + 1]].tolist()) for i in range(A.n)]


@pytest.mark.parametrize("maker", [lambda: poisson2d(12), lambda: poisson3d(6), lambda: varcoef3d(6, 1.0, 2, 100.0)[0],
                                   lambda: random_csr(60, 5, 7, symmetric=True)])
def test_rs_first_pass_structure(oracle_lib, maker):
    """Brute-force structural facts of the RS first pass: every F point with a strong connection has a
    strong C point; for a symmetric strength graph no C point strongly depends on another C point."""
    O = oracle_lib
    A = maker()
    cf = O.coarsen(A, 0.25)
    S = _strong_sets(O, A, 0.25)
    ST = [set() for _ in range(A.n)]
    for i, s in enumerate(S):
        for j in s:
            ST[j].add(i)
    for i in range(A.n):
        if cf[i] == 0 and (S[i] or ST[i]):
            assert any(cf[j] == 1 for j in S[i]), i
    if all(S[i] == {j for j in range(A.n) if i in S[j]} for i in range(A.n)):
        for i in range(A.n):
            if cf[i] == 1:
                assert not any(cf[j] == 1 for j in S[i])
    assert 0 < cf.sum() < A.n


def test_rs_tie_break_smallest_index(oracle_lib):
    """Equal measures: the smallest index is chosen first. On a 5-point 3x3 grid the corner 0 and the
    centre 4 both have measure... the centre has the largest measure (4) and becomes C first."""
    cf = oracle_lib.coarsen(poisson2d(3), 0.25)
    # centre 4 (measure 4) -> C, its 4 neighbours F; the corners then have measure 4 (two F neighbours):
    # all corners become C in index order.
    assert list(cf) == [1, 0, 1, 0, 1, 0, 1, 0, 1]


def _graph_matrix(n, edges):
    """Symmetric matrix with -1 on every edge and degree + 1 on the diagonal (isolated points: 1)."""
    d = np.zeros((n, n))
    for i, j in edges:
        d[i, j] = d[j, i] = -1.0
    np.fill_diagonal(d, np.abs(d).sum(axis=1) + 1.0)
    return CSR.from_dense(d)


def _rs_by_definition(n, edges, f_weight=2, largest_first=False):
    """The first pass written from its definition for a symmetric graph: recompute every measure from
    scratch after each decision (tiny inputs only)."""
    nb = [set() for _ in range(n)]
    for i, j in edges:
        nb[i].add(j)
        nb[j].add(i)
    state = ["F" if not nb[i] else "U" for i in range(n)]
    while "U" in state:
        lam = {i: sum(1 if state[j] == "U" else (f_weight if state[j] == "F" else 0) for j in nb[i])
               for i in range(n) if state[i] == "U"}
        top = max(lam.values())
        ties = [i for i in sorted(lam) if lam[i] == top]
        i = ties[-1] if largest_first else ties[0]
        state[i] = "C"
        for j in nb[i]:
            if state[j] == "U":
                state[j] = "F"
    return [1 if s == "C" else 0 for s in state]


def test_rs_first_pass_hand_worked_golden(oracle_lib):
    """Hand-worked RS first passes (tests/golden/rs_first_pass_hand.json): tridiag(4) fixes the
    smallest-index tie-break (C = {1, 3}, not {0, 2}); the 11-point graph fixes the weight 2 on F
    dependents (a weight of 1 or 0, or the largest-index tie-break, gives a different splitting)."""
    g = json.load(open(os.path.join(GOLD, "rs_first_pass_hand.json")))
    for case in g["cases"]:
        A = _graph_matrix(case["n"], case["edges"])
        cf = list(oracle_lib.coarsen(A, g["theta"]))
        assert cf == case["cf"], case["name"]
        # the golden's alternatives really differ, so the pin discriminates those readings
        assert case["cf_if_largest_index_first"] != case["cf"]
        assert _rs_by_definition(case["n"], case["edges"], largest_first=True) == case["cf_if_largest_index_first"]
        assert _rs_by_definition(case["n"], case["edges"]) == case["cf"]
        if "cf_if_f_weight_1" in case:
            assert case["cf_if_f_weight_1"] != case["cf"]
            assert _rs_by_definition(case["n"], case["edges"], f_weight=1) == case["cf_if_f_weight_1"]
            assert _rs_by_definition(case["n"], case["edges"], f_weight=0) == case["cf_if_f_weight_1"]


@pytest.mark.parametrize("seed", range(40))
def test_rs_first_pass_matches_definition_on_random_graphs(oracle_lib, seed):
    """The incremental first pass of the oracle against the definition (every measure recomputed after
    each decision) on random symmetric graphs of 6-30 points with isolated points and ties."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 31))
    p = float(rng.uniform(0.08, 0.4))
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    A = _graph_matrix(n, edges)
    assert list(oracle_lib.coarsen(A, 0.25)) == _rs_by_definition(n, edges)


# ------------------------------------------------------------------------------ interpolation / RAP
@pytest.mark.parametrize("maker", [lambda: poisson2d(16), lambda: poisson3d(8), lambda: varcoef3d(8, 1.0, 2, 100.0)[0]])
def test_classical_interp_preserves_constants(oracle_lib, maker):
    """Classical interpolation reproduces constants on every row whose A-row sums to zero (the identity
    sum_j w_ij = 1 follows from den_k = sum_{l in C_i} a_kl and a zero row sum)."""
    A = maker()
    H = oracle_lib.Hierarchy(A, max_levels=2, max_coarse=1)
    L0 = H.level(0)
    rowsum = A.to_scipy() @ np.ones(A.n)
    p1 = L0.P @ np.ones(L0.P.shape[1])
    zero_rows = np.abs(rowsum) < 1e-12 * np.abs(A.vals).max()
    assert zero_rows.sum() > 0
    np.testing.assert_allclose(p1[zero_rows], 1.0, atol=1e-14)
    assert np.all(p1[L0.cf == 1] == 1.0)


@pytest.mark.parametrize("maker", [lambda: poisson2d(20), lambda: poisson3d(8), lambda: convdiff3d(7, 3)[0]])
def test_galerkin_matches_scipy_triple_product(oracle_lib, maker):
    """Section 5: A_{k+1} = P^T A_k P. Compared with scipy's sparse triple product on every level."""
    A = maker()
    H = oracle_lib.Hierarchy(A, max_coarse=10)
    assert H.levels >= 3
    for l in range(H.levels - 1):
        L = H.level(l)
        Ac = H.level(l + 1).A
        ref = (L.P.T @ L.A.to_scipy() @ L.P).toarray()
        got = Ac.to_dense()
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        # stored pattern covers every nonzero of the product
        assert np.all((ref != 0) <= (got != 0) | (np.abs(ref) < 1e-15))


def test_galerkin_symmetric_for_symmetric_A(oracle_lib):
    H = oracle_lib.Hierarchy(varcoef3d(8, 1.0, 2, 100.0)[0], max_coarse=10)
    for l in range(1, H.levels):
        d = H.level(l).A.to_dense()
        assert np.abs(d - d.T).max() <= 1e-14 * np.abs(d).max()


# ------------------------------------------------------------------------------------------ ILU(0)
def _split_ilu(A, w):
    n = A.n
    L, U = np.eye(n), np.zeros((n, n))
    for i in range(n):
        for k in range(A.rowptr[i], A.rowptr[i + 1]):
            j = A.colind[k]
            (L if j < i else U)[i, j] = w[k]
    return L, U


@pytest.mark.parametrize("maker", [lambda: poisson2d(8), lambda: convdiff3d(4, 3)[0], lambda: random_csr(30, 5, 3)])
def test_ilu0_reproduces_A_on_pattern(oracle_lib, maker):
    """ILU(0) (Chow & Saad, Section 1): (LU)_ij = a_ij at every position of A's pattern."""
    A = maker()
    L, U = _split_ilu(A, oracle_lib.ilu0(A))
    LU = L @ U
    Ad = A.to_dense()
    mask = Ad != 0
    np.testing.assert_allclose(LU[mask], Ad[mask], atol=1e-13)


def test_ilu0_tridiagonal_is_exact_lu(oracle_lib):
    """No fill for tridiagonal A, so ILU(0) = LU and the ILU-direct sweep solves A x = b exactly."""
    A = tridiag1d(25)
    L, U = _split_ilu(A, oracle_lib.ilu0(A))
    np.testing.assert_allclose(L @ U, A.to_dense(), atol=1e-14)
    b = np.random.default_rng(4).standard_normal(A.n)
    x = oracle_lib.smooth(A, oracle_lib.ILU_DIRECT, 1, b, np.zeros(A.n))
    np.testing.assert_allclose(x, np.linalg.solve(A.to_dense(), b), rtol=1e-12)


# -------------------------------------------------------------------------------------------- ILUT
def _split_factor(F):
    """Dense (L, U) from a CSR holding L \\ U (unit diagonal of L implied)."""
    d = F.to_dense()
    return np.tril(d, -1) + np.eye(F.n), np.triu(d)


@pytest.mark.parametrize("maker", [lambda: poisson2d(6), lambda: convdiff3d(3, 3)[0], lambda: random_csr(30, 5, 3)])
def test_ilut_without_dropping_is_exact_lu(oracle_lib, maker):
    """ILUT with droptol = 0 and no fill limit drops nothing, so it is Gaussian elimination without
    pivoting: the LU factors scipy computes (whose partial pivoting picks the diagonal on these
    diagonally dominant matrices), and one direct sweep from x = 0 solves A x = b."""
    O = oracle_lib
    A = maker()
    F = O.ilut(A, 0.0, A.n)
    L, U = _split_factor(F)
    P, Ls, Us = sla.lu(A.to_dense())
    assert np.array_equal(P, np.eye(A.n))
    np.testing.assert_allclose(L, Ls, atol=1e-13)
    np.testing.assert_allclose(U, Us, atol=1e-12)
    b = np.random.default_rng(1).standard_normal(A.n)
    x = O.smooth_ilut(A, 0.0, A.n, 1, b, np.zeros(A.n), direct=True)
    np.testing.assert_allclose(x, np.linalg.solve(A.to_dense(), b), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("droptol", [1e-3, 1e-2, 1e-1])
@pytest.mark.parametrize("maker", [lambda: poisson2d(10), lambda: convdiff3d(4, 3)[0], lambda: random_csr(40, 6, 2)])
def test_ilut_reproduces_A_on_its_pattern(oracle_lib, maker, droptol):
    """Without the fill limit every multiplier ILUT keeps is used and stored, and every stored U entry is
    the one later rows eliminate with, so (LU)_ij = a_ij at each stored position; a position of A that
    is not stored was dropped at the end of its row, so there LU differs from A by less than the
    row's threshold droptol ||a_i||_2 (times u_jj for a lower entry)."""
    O = oracle_lib
    A = maker()
    F = O.ilut(A, droptol, A.n)
    L, U = _split_factor(F)
    Ad, LU = A.to_dense(), L @ U
    mask = F.to_dense() != 0
    np.testing.assert_allclose(LU[mask], Ad[mask], atol=1e-12 * np.abs(Ad).max())
    tau = droptol * np.linalg.norm(Ad, axis=1)
    ii, jj = np.nonzero((Ad != 0) & ~mask)
    bound = np.where(jj < ii, tau[ii] * np.abs(np.diag(U))[jj], tau[ii])
    assert np.all(np.abs(LU[ii, jj] - Ad[ii, jj]) <= bound * (1 + 1e-12))


def test_ilut_degenerate_limits(oracle_lib):
    """A drop tolerance above every entry, or lfil = 0, leaves only the diagonal: with no stored U rows
    nothing updates u_ii, so U = diag(A) and the Neumann ILUT sweep is a Jacobi step x + D^{-1}(b - A x)."""
    O = oracle_lib
    A = poisson2d(7)
    Ad = A.to_dense()
    for F in (O.ilut(A, 1e3, 5), O.ilut(A, 1e-2, 0)):
        np.testing.assert_array_equal(F.to_dense(), np.diag(np.diag(Ad)))
    rng = np.random.default_rng(2)
    b, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    jac = x + (b - Ad @ x) / np.diag(Ad)
    np.testing.assert_allclose(O.smooth_ilut(A, 1e-2, 0, 3, b, x), jac, rtol=1e-14, atol=1e-14)


def test_ilut_keeps_the_lfil_largest(oracle_lib):
    """Row 0 has nothing to eliminate, so U's row 0 is A's row 0 after the two rules: entries below
    droptol * ||a_0||_2 go, then the lfil largest in magnitude stay (equal magnitudes: smaller column)."""
    O = oracle_lib
    d = np.eye(8) * 10.0
    d[0, 1:] = [-1.0, 1.0, -1.0, 0.5, 3.0, 0.01, -1.0]
    d[1:, 0] = 0.1
    A = CSR.from_dense(d)
    F = O.ilut(A, 0.05 / np.linalg.norm(d[0]), 3)  # tau = 0.05: drops the 0.01 entry
    row0 = F.to_dense()[0]
    assert list(np.nonzero(row0[1:])[0] + 1) == [1, 2, 5]  # 3.0, then the first two of the four |1|
    assert row0[5] == 3.0 and row0[1] == -1.0 and row0[2] == 1.0
    F = O.ilut(A, 0.0, 7)
    np.testing.assert_array_equal(F.to_dense()[0], d[0])
    F = O.ilut(A, 0.05 / np.linalg.norm(d[0]), 7)
    assert F.to_dense()[0, 6] == 0.0 and np.count_nonzero(F.to_dense()[0]) == 7
    # tau = 0.9 in the row's 2-norm drops 0.5 and 0.01 but none of the |1| (the 1-norm would drop them)
    F = O.ilut(A, 0.9 / np.linalg.norm(d[0]), 7)
    assert list(np.nonzero(F.to_dense()[0])[0]) == [0, 1, 2, 3, 5, 7]


def test_ilut_fill_limits_and_tridiagonal(oracle_lib):
    """At most lfil entries per row in each strict triangle; on a tridiagonal matrix there is no fill,
    so ILUT(0, 1) is ILU(0), the exact LU."""
    O = oracle_lib
    A = poisson2d(16)
    for droptol, lfil in ((1e-2, 5), (1e-3, 2), (0.0, 1)):
        F = O.ilut(A, droptol, lfil)
        for i in range(A.n):
            cols = F.colind[F.rowptr[i]:F.rowptr[i + 1]]
            assert (cols < i).sum() <= lfil and (cols > i).sum() <= lfil and i in cols
            assert np.all(np.diff(cols) > 0)
    T = tridiag1d(20)
    F = O.ilut(T, 0.0, 1)
    np.testing.assert_array_equal(F.rowptr, T.rowptr)
    np.testing.assert_array_equal(F.colind, T.colind)
    np.testing.assert_allclose(F.vals, O.ilu0(T), rtol=1e-15)


def test_ilut_hierarchy_solves(oracle_lib):
    """The hybrid V-cycle with ILUT(1e-2, 5) on the finest level (Algorithm 2 with row scaling) as
    preconditioner: converges to the true relative residual with Jacobi and with direct triangular
    solves, and the direct ILUT smoother needs no more iterations than the direct ILU(0) one."""
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c2", 12)
    H = O.Hierarchy(A, ilu_kind=O.ILU_KIND_ILUT, ilut_droptol=1e-2, ilut_lfil=5)
    H0 = O.Hierarchy(A)
    Ad = A.to_dense()
    for tri in (O.TRI_NEUMANN, O.TRI_DIRECT):
        r = H.solve(b, smoother=O.SMOOTH_ILU0, tri_mode=tri, t=3)
        assert r["status"] == 0 and np.linalg.norm(b - Ad @ r["x"]) <= 1e-8 * np.linalg.norm(b)
    assert (H.solve(b, smoother=O.SMOOTH_ILU0, tri_mode=O.TRI_DIRECT)["iters"]
            <= H0.solve(b, smoother=O.SMOOTH_ILU0, tri_mode=O.TRI_DIRECT)["iters"])
    with pytest.raises(O.OracleFailure):
        O.Hierarchy(A, ilu_kind=O.ILU_KIND_ILUT, ilut_lfil=-1)
    with pytest.raises(O.OracleFailure):
        O.Hierarchy(A, ilu_kind=2)


# ---------------------------------------------------------------------------------------- smoothers
def _depth(A, lower=True):
    """Number of levels of the dependency DAG of the strict triangle (brute force)."""
    lev = np.zeros(A.n, int)
    order = range(A.n) if lower else range(A.n - 1, -1, -1)
    for i in order:
        cols = A.colind[A.rowptr[i]:A.rowptr[i + 1]]
        dep = cols[cols < i] if lower else cols[cols > i]
        lev[i] = 1 + (lev[dep].max() if dep.size else 0)
    return lev.max()


def test_pgs_zero_inner_sweeps_is_jacobi(oracle_lib):
    """Section 5.2: with zero inner sweeps polynomial GS is the Jacobi iteration x + D^{-1}(b - A x)."""
    A = varcoef3d(5, 1.0, 2, 100.0)[0]
    rng = np.random.default_rng(1)
    b, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    Ad = A.to_dense()
    ref = x + (b - Ad @ x) / np.diag(Ad)
    for kind in (oracle_lib.PGS_FWD, oracle_lib.PGS_BWD):
        np.testing.assert_allclose(oracle_lib.smooth(A, kind, 1, b, x), ref, rtol=1e-13)


def test_gs_direct_is_triangular_solve(oracle_lib):
    A = convdiff3d(4, 3)[0]
    rng = np.random.default_rng(2)
    b, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    Ad = A.to_dense()
    r = b - Ad @ x
    fw = x + sla.solve_triangular(np.tril(Ad), r, lower=True)
    bw = x + sla.solve_triangular(np.triu(Ad), r, lower=False)
    np.testing.assert_allclose(oracle_lib.smooth(A, oracle_lib.GS_FWD, 1, b, x), fw, rtol=1e-12)
    np.testing.assert_allclose(oracle_lib.smooth(A, oracle_lib.GS_BWD, 1, b, x), bw, rtol=1e-12)


def test_neumann_terminates_at_dependency_depth(oracle_lib):
    """Section 5.2 / 5.3.2: D^{-1}L and U_s are nilpotent, so the Neumann series is finite. For the
    8x8 5-point grid the lower triangle has depth 15: 15 terms reproduce the forward substitution,
    14 terms do not. The same holds for ILU(0) with its L_s and U_s."""
    O = oracle_lib
    A = poisson2d(8)
    assert _depth(A, True) == 15 and _depth(A, False) == 15
    rng = np.random.default_rng(3)
    b, x = rng.standard_normal(A.n), np.zeros(A.n)
    ref = O.smooth(A, O.GS_FWD, 1, b, x)
    e15 = np.abs(O.smooth(A, O.PGS_FWD, 15, b, x) - ref).max() / np.abs(ref).max()
    e14 = np.abs(O.smooth(A, O.PGS_FWD, 14, b, x) - ref).max() / np.abs(ref).max()
    assert e15 < 1e-15 and e14 > 1e-9
    refb = O.smooth(A, O.GS_BWD, 1, b, x)
    assert np.abs(O.smooth(A, O.PGS_BWD, 15, b, x) - refb).max() < 1e-15 * np.abs(refb).max() * 10
    ref_ilu = O.smooth(A, O.ILU_DIRECT, 1, b, x)
    e_ilu15 = np.abs(O.smooth(A, O.ILU_NEUMANN, 15, b, x) - ref_ilu).max() / np.abs(ref_ilu).max()
    e_ilu14 = np.abs(O.smooth(A, O.ILU_NEUMANN, 14, b, x) - ref_ilu).max() / np.abs(ref_ilu).max()
    assert e_ilu15 < 1e-14 and e_ilu14 > 1e-12


def test_ilu_neumann_is_truncated_series(oracle_lib):
    """Section 5.3.2, eq. (Neumann): with L = I + L_s and U = D_U (I + U_s) the t-term sweep applies
    (sum_{j<t} (-U_s)^j) D_U^{-1} (sum_{j<t} (-L_s)^j) to the residual. Checked with dense powers."""
    O = oracle_lib
    A = convdiff3d(4, 3)[0]
    L, U = _split_ilu(A, O.ilu0(A))
    Ls = L - np.eye(A.n)
    Du = np.diag(np.diag(U))
    Us = np.linalg.solve(Du, U) - np.eye(A.n)
    rng = np.random.default_rng(5)
    b, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    r = b - A.to_dense() @ x
    for t in (1, 2, 3, 5):
        NL = sum(np.linalg.matrix_power(-Ls, j) for j in range(t))
        NU = sum(np.linalg.matrix_power(-Us, j) for j in range(t))
        ref = x + NU @ np.linalg.solve(Du, NL @ r)
        np.testing.assert_allclose(O.smooth(A, O.ILU_NEUMANN, t, b, x), ref, rtol=1e-11, atol=1e-12)


def test_numerical_nilpotence_of_ilu_factor(oracle_lib):
    """Section 5.3.2 (Figure 1's phenomenon): ||U_s^p|| decays long before p = n and is exactly zero
    at p = dependency depth, on the ILU(0) factor of a nonsymmetric 3-D operator."""
    A = convdiff3d(5, 3)[0]
    L, U = _split_ilu(A, oracle_lib.ilu0(A))
    Us = np.triu(U / np.diag(U)[:, None], 1)  # D_U^{-1} U = I + U_s
    d = _depth(A, False)
    assert d < A.n
    norms = [np.linalg.norm(np.linalg.matrix_power(Us, p), 2) for p in (1, 4, 8, d - 1, d)]
    assert norms[0] < 1.0 and norms[2] < 0.05 * norms[0]
    assert norms[-2] > 0 and norms[-1] == 0.0


# ----------------------------------------------------------------------------------------- V-cycle
def test_one_level_hierarchy_is_direct_solve(oracle_lib):
    A = poisson2d(6)  # n = 36 <= max_coarse
    H = oracle_lib.Hierarchy(A)
    assert H.levels == 1
    b = np.random.default_rng(0).standard_normal(A.n)
    np.testing.assert_allclose(H.vcycle(b), np.linalg.solve(A.to_dense(), b), rtol=1e-13)


def test_l1_jacobi_closed_forms(oracle_lib):
    """l1-Jacobi, x <- x + D_l1^{-1}(b - A x) with (D_l1)_ii = sum_j |a_ij| (the Table 6 comparator):
    one sweep from x = 0 on the 5-point Poisson matrix is x_i = b_i / (4 + number of neighbours of i);
    on a positive diagonal matrix one sweep is the exact solve; repeated sweeps converge to A^{-1} b
    (D_l1 - A is positive semidefinite for symmetric A with positive diagonal, so the iteration
    contracts in the A-norm)."""
    O = oracle_lib
    N = 6
    A = poisson2d(N)
    b = np.random.default_rng(2).standard_normal(A.n)
    x1 = O.smooth(A, O.L1_JACOBI, 1, b, np.zeros(A.n))
    gx, gy = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    nb = (gx > 0).astype(int) + (gx < N - 1) + (gy > 0) + (gy < N - 1)
    np.testing.assert_allclose(x1, b / (4.0 + nb.ravel()), rtol=1e-15)
    dvals = np.linspace(1.0, 5.0, 9)
    D = CSR.from_dense(np.diag(dvals))
    np.testing.assert_allclose(O.smooth(D, O.L1_JACOBI, 1, dvals * 2.0, np.ones(9)), 2.0 * np.ones(9), rtol=1e-15)
    xs = np.linalg.solve(A.to_dense(), b)
    x = np.zeros(A.n)
    errs = []
    for _ in range(400):
        x = O.smooth(A, O.L1_JACOBI, 1, b, x)
        e = x - xs
        errs.append(np.sqrt(e @ (A.to_dense() @ e)))
    assert all(e2 <= e1 * (1 + 1e-12) for e1, e2 in zip(errs, errs[1:]))
    np.testing.assert_allclose(x, xs, rtol=1e-8, atol=1e-10)


def test_l1_jacobi_preconditioned_solve(oracle_lib):
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c1")
    r = O.Hierarchy(A).solve(b, smoother=O.SMOOTH_L1JAC)
    assert r["status"] == 0 and r["relres_true"] <= 1e-8


def _dense_op(f, n):
    return np.stack([f(e) for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("smoother,tri", [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0)])
def test_vcycle_linear_and_symmetric(oracle_lib, smoother, tri):
    """The V-cycle is a linear operator; with forward pre- and backward post-smoothing (PGS), the ILU
    sweep (symmetric A gives U = D L^T) or l1-Jacobi (a symmetric smoother) it is symmetric for
    symmetric A."""
    O = oracle_lib
    A = poisson2d(10)
    H = O.Hierarchy(A, ilu_levels=1)
    assert H.levels >= 2
    M = _dense_op(lambda e: H.vcycle(e, smoother=smoother, tri_mode=tri, t=3), A.n)
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    rng = np.random.default_rng(6)
    u, v = rng.standard_normal(A.n), rng.standard_normal(A.n)
    lhs = H.vcycle(2.0 * u - 3.0 * v, smoother=smoother, tri_mode=tri, t=3)
    np.testing.assert_allclose(lhs, M @ (2.0 * u - 3.0 * v), rtol=1e-12, atol=1e-14)


def test_two_grid_coarse_correction_is_galerkin_projection(oracle_lib):
    """With no smoothing and an exact coarse solve the V-cycle on two levels is P (P^T A P)^{-1} P^T,
    the Galerkin coarse-grid correction (Section 5)."""
    O = oracle_lib
    A = poisson2d(9)
    H = O.Hierarchy(A, max_levels=2)
    assert H.levels == 2
    P = H.level(0).P.toarray()
    Ad = A.to_dense()
    ref = P @ np.linalg.solve(P.T @ Ad @ P, P.T)
    M = _dense_op(lambda e: H.vcycle(e, nu1=0, nu2=0), A.n)
    np.testing.assert_allclose(M, ref, atol=1e-13)


# ------------------------------------------------------------------------------------------- GMRES
def test_gmres_terminates_at_number_of_distinct_eigenvalues(oracle_lib):
    """4x4 5-point Poisson has 9 distinct eigenvalues: unpreconditioned GMRES with a generic b reaches
    the exact solution at iteration 9 and not before (Krylov space dimension), for both T forms."""
    O = oracle_lib
    A = poisson2d(4)
    b = np.random.default_rng(0).standard_normal(A.n)
    H = O.Hierarchy(A)
    for T in (O.T_NEUMANN, O.T_DIRECT):
        r = H.solve(b, tol=1e-13, restart=16, precond=O.PRECOND_NONE, gmres_T=T)
        assert r["iters"] == 9 and r["status"] == 0
        assert r["hist"][7] > 1e-6 and r["hist"][8] < 1e-13
        assert r["relres_true"] < 1e-13


def test_gmres_ritz_values_are_poisson_eigenvalues(oracle_lib):
    O = oracle_lib
    A = poisson2d(4)
    b = np.random.default_rng(1).standard_normal(A.n)
    r = O.Hierarchy(A).solve(b, tol=1e-14, restart=16, max_iters=9, precond=O.PRECOND_NONE, capture=True)
    k = r["k"]
    assert k == 9
    ritz = np.sort(np.linalg.eigvals(r["H"][:k, :k]).real)
    c = np.cos(np.arange(1, 5) * np.pi / 5)
    lam = np.unique(np.round(4 - 2 * (c[:, None] + c[None, :]), 12))
    np.testing.assert_allclose(ritz, np.sort(lam), atol=1e-10)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_gmres_iterate_is_krylov_least_squares(oracle_lib, k):
    """GMRES (Section 1): x_k minimises ||b - A x|| over x0 + K_k(A, r0). Dense least squares on an
    orthonormal basis of the Krylov space (numpy QR + lstsq) gives the same x_k."""
    O = oracle_lib
    A = random_csr(30, 5, 11)
    Ad = A.to_dense()
    rng = np.random.default_rng(2)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    res = O.Hierarchy(A, max_coarse=100).solve(b, x0, tol=1e-15, restart=30, max_iters=k,
                                               precond=O.PRECOND_NONE)
    r0 = b - Ad @ x0
    K = np.stack([np.linalg.matrix_power(Ad, j) @ r0 for j in range(k)], axis=1)
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(Ad @ Q, r0, rcond=None)
    np.testing.assert_allclose(res["x"], x0 + Q @ y, rtol=1e-10, atol=1e-12)


def test_flexible_gmres_with_fixed_amg_minimises_over_MK(oracle_lib):
    """Right preconditioning with a fixed linear M: x_k minimises the residual over x0 + M K_k(A M, r0)."""
    O = oracle_lib
    A = poisson2d(9)
    Ad = A.to_dense()
    H = O.Hierarchy(A)
    M = _dense_op(lambda e: H.vcycle(e, t=2), A.n)
    b = np.random.default_rng(3).standard_normal(A.n)
    for k in (1, 2, 3):
        res = H.solve(b, tol=1e-15, restart=30, max_iters=k, t=2)
        AM = Ad @ M
        K = np.stack([np.linalg.matrix_power(AM, j) @ b for j in range(k)], axis=1)
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(AM @ Q, b, rcond=None)
        np.testing.assert_allclose(res["x"], M @ Q @ y, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("T", [0, 1])
@pytest.mark.parametrize("tol", [1e-8, 1e-12])
def test_arnoldi_relation_and_orthogonality(oracle_lib, T, tol):
    """A Z_k = V_{k+1} H_{k+1,k} (flexible Arnoldi, Section 1) to rounding, and the loss of orthogonality
    ||I - V^T V||_F stays below O(eps) kappa(B), B = [r0, A Z_k] with unit columns (Section 3)."""
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c1")
    r = O.Hierarchy(A).solve(b, tol=tol, restart=30, t=2, gmres_T=T, capture=True)
    V, Z, Hh, k = r["V"], r["Z"], r["H"], r["k"]
    AZ = A.to_scipy() @ Z
    assert np.linalg.norm(AZ - V @ Hh) / np.linalg.norm(AZ) < 1e-14
    B = np.column_stack([b, AZ])
    sv = np.linalg.svd(B / np.linalg.norm(B, axis=0), compute_uv=False)
    kappa = sv[0] / sv[-1]
    loo = O.loss_orth(V)
    assert loo <= 10.0 * np.finfo(float).eps * kappa
    # Section 3: beta(x) kappa(B) = O(1) -- the orthogonality loss grows as the backward error falls
    assert r["nrbe"] * kappa < 100.0


def test_T_neumann_matches_T_direct(oracle_lib):
    """Section 1/3: the truncated T = I - L gives the same convergence history as (I + L)^{-1}."""
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c1")
    H = O.Hierarchy(A)
    a = H.solve(b, t=2, gmres_T=O.T_NEUMANN)
    c = H.solve(b, t=2, gmres_T=O.T_DIRECT)
    assert a["iters"] == c["iters"]
    np.testing.assert_allclose(a["hist"], c["hist"], rtol=1e-8)
    np.testing.assert_allclose(a["x"], c["x"], rtol=1e-12, atol=1e-12 * np.abs(c["x"]).max())
    assert a["relres_true"] <= 1e-8


def _ill_conditioned_dense(n=60, seed=7):
    """A dense nonsymmetric matrix with singular values logspace(0, 8): unpreconditioned GMRES loses
    orthogonality quickly on it, so the lower triangle L of the low-sync step is far from negligible."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    W, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (U * np.logspace(0, 8, n)) @ W.T
    return CSR.from_dense(A), rng.standard_normal(n)


def test_t_degree_one_is_I_minus_L(oracle_lib):
    """Degree p = 1 of T = sum_{j<=p} (-L)^j is the default T = I - L, bit for bit."""
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c1")
    H = O.Hierarchy(A)
    a = H.solve(b, t=2)
    c = H.solve(b, t=2, t_degree=1)
    assert a["iters"] == c["iters"] and np.array_equal(a["x"], c["x"])


def test_t_degree_truncation_error(oracle_lib):
    """Section 1: T = sum_{j<=p} (-L)^j truncates the Neumann series of (I + L)^{-1}, with an error of
    order ||L||^(p+1). Where L is far from negligible (loss of orthogonality near 1 after 60 steps),
    p = 1 differs visibly from the exact (I + L)^{-1}, p = 2 already agrees to rounding, and p >= the
    step count is exact because L is nilpotent."""
    O = oracle_lib
    A, b = _ill_conditioned_dense()
    H = O.Hierarchy(A, max_coarse=A.n + 1)
    kw = dict(precond=O.PRECOND_NONE, restart=60, max_iters=60, tol=1e-14, capture=True)
    d = H.solve(b, gmres_T=O.T_DIRECT, **kw)
    assert O.loss_orth(d["V"]) > 0.5
    err = {}
    for p in (1, 2, 3, 60):
        r = H.solve(b, gmres_T=O.T_NEUMANN, t_degree=p, **kw)
        assert r["iters"] == d["iters"]
        err[p] = np.linalg.norm(r["x"] - d["x"]) / np.linalg.norm(d["x"])
    assert err[1] > 1e-12
    assert err[2] <= 1e-14 and err[3] <= 1e-14 and err[60] <= 1e-14
    with pytest.raises(O.OracleFailure):
        H.solve(b, t_degree=0)


def test_nrbe_stopping_rule(oracle_lib):
    """Section 3: stopping on the normwise relative backward error ||r|| / (||b|| + ||A||_inf ||x||).
    The solve ends with NRBE <= tol; since NRBE <= ||r|| / ||b|| at any x, the rule never takes more
    iterations than the relative-residual rule. Inside a cycle the denominator uses the cycle's
    starting iterate, so the first cycle (x0 = 0) stops where the relative-residual rule does; with
    short restarts later cycles see ||A||_inf ||x|| >> ||b|| and stop strictly earlier. The rule
    only changes when the iteration stops: its iterate equals the relative-residual run cut off at
    the same iteration count."""
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c1")
    H = O.Hierarchy(A)
    rel = H.solve(b, tol=1e-8, t=2)
    nrbe = H.solve(b, tol=1e-8, t=2, stop_rule=O.STOP_NRBE)
    assert nrbe["status"] == 0 and nrbe["nrbe"] <= 1e-8
    Ad = A.to_dense()
    r = b - Ad @ nrbe["x"]
    direct = np.linalg.norm(r) / (np.linalg.norm(b) + np.abs(Ad).sum(axis=1).max() * np.linalg.norm(nrbe["x"]))
    assert nrbe["nrbe"] == pytest.approx(direct, rel=1e-6)
    assert nrbe["iters"] <= rel["iters"]
    for rhs in (b, np.ones(A.n)):
        short_rel = H.solve(rhs, tol=1e-8, t=2, restart=3)
        short = H.solve(rhs, tol=1e-8, t=2, restart=3, stop_rule=O.STOP_NRBE)
        assert short["status"] == 0 and short["iters"] < short_rel["iters"]
        cut = H.solve(rhs, tol=1e-8, t=2, restart=3, max_iters=short["iters"])
        assert cut["iters"] == short["iters"]
        np.testing.assert_array_equal(cut["x"], short["x"])
    with pytest.raises(O.OracleFailure):
        H.solve(b, stop_rule=2)


def test_lucky_breakdown_on_eigenvector(oracle_lib):
    O = oracle_lib
    N = 7
    g = np.arange(1, N + 1) / (N + 1)
    v = np.outer(np.sin(2 * np.pi * g), np.sin(np.pi * g)).ravel()
    lam = 4 - 2 * np.cos(np.pi / (N + 1)) - 2 * np.cos(2 * np.pi / (N + 1))
    r = O.Hierarchy(poisson2d(N)).solve(v, tol=1e-12, precond=O.PRECOND_NONE)
    assert r["status"] == 0 and r["iters"] == 1
    np.testing.assert_allclose(r["x"], v / lam, rtol=1e-13)


def test_restarted_gmres_and_nrbe(oracle_lib):
    """Small restart still converges on the true residual; the NRBE of Section 3 is
    ||r|| / (||b|| + ||A||_inf ||x||)."""
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c1")
    r = O.Hierarchy(A).solve(b, tol=1e-8, restart=3, t=2)
    assert r["status"] == 0 and r["cycles"] > 1 and r["relres_true"] <= 1e-8
    Ad = A.to_dense()
    res = np.linalg.norm(b - Ad @ r["x"])
    nrbe = res / (np.linalg.norm(b) + np.abs(Ad).sum(1).max() * np.linalg.norm(r["x"]))
    assert abs(r["nrbe"] - nrbe) <= 1e-6 * nrbe
    assert abs(r["relres_true"] - res / np.linalg.norm(b)) <= 1e-6 * r["relres_true"]


def test_not_converged_status_and_error_paths(oracle_lib):
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c1")
    H = O.Hierarchy(A)
    r = H.solve(b, tol=1e-20, max_iters=2, t=2)
    assert r["status"] == O.NOT_CONVERGED and r["iters"] == 2
    bad = b.copy()
    bad[3] = np.nan
    with pytest.raises(O.OracleFailure) as e:
        H.solve(bad)
    assert e.value.code == O.E_NONFINITE
    d = A.to_dense()
    d[5, 5] = 0.0
    with pytest.raises(O.OracleFailure) as e:
        O.Hierarchy(CSR.from_dense(d))
    assert e.value.code == O.E_ZERO_PIVOT
    Z = CSR(A.n, A.rowptr, A.colind.copy(), A.vals)
    Z.colind[[0, 1]] = Z.colind[[1, 0]]
    with pytest.raises(O.OracleFailure) as e:
        O.Hierarchy(Z)
    assert e.value.code == O.E_INVALID


# ------------------------------------------------------------ non-normality (Sections 5.3.1 to 5.3.4)
def test_henrici_departure_closed_forms():
    """dep(T)^2 = ||T||_F^2 - sum |lambda|^2: zero for normal matrices, |a| for [[1, a], [0, 2]], and
    ||strict(T)||_F for any triangular T (its eigenvalues are its diagonal)."""
    from oracle.nonnormal import henrici_dep

    assert henrici_dep(np.array([[1.0, -3.5], [0.0, 2.0]])) == pytest.approx(3.5, rel=1e-14)
    rng = np.random.default_rng(3)
    S = rng.standard_normal((30, 30))
    S = S + S.T
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    for N in (S, Q):
        assert henrici_dep(N) <= 1e-6 * np.linalg.norm(N, "fro")
    T = np.triu(rng.standard_normal((40, 40)))
    assert henrici_dep(T) == pytest.approx(np.linalg.norm(np.triu(T, 1), "fro"), rel=1e-10)


def test_ruiz_equilibrates_rows_and_columns():
    """Ruiz scaling converges to a matrix whose every row and column has largest magnitude 1 (to tol);
    a symmetric matrix gets equal row and column scalings; a diagonal matrix becomes I in one step."""
    from oracle.nonnormal import ruiz

    A = random_csr(60, 6, 5).to_dense()
    U = np.triu(A) * np.exp(np.random.default_rng(1).uniform(-6, 6, 60))[:, None]  # badly row-scaled
    dr, dc, it = ruiz(U, 1e-10, 100)
    S = np.abs(dr[:, None] * U * dc[None, :])
    assert 1 <= it < 100
    np.testing.assert_allclose(S.max(axis=1), 1.0, atol=1e-10)
    np.testing.assert_allclose(S.max(axis=0), 1.0, atol=1e-10)
    As = A + A.T
    dr, dc, _ = ruiz(As, 1e-12, 100)
    np.testing.assert_array_equal(dr, dc)
    D = np.diag(np.arange(1.0, 9.0) ** 3)
    dr, dc, it = ruiz(D, 1e-14, 10)
    assert it == 1
    np.testing.assert_allclose(dr[:, None] * D * dc[None, :], np.eye(8), atol=1e-15)


@pytest.mark.parametrize("droptol,lfil", [(1e-2, 5), (1e-3, 10), (1e-1, 2)])
def test_theorems_1_to_4_hold_on_ilut_factors(oracle_lib, droptol, lfil):
    """Section 5.3.4 on ILUT factors of a nonsymmetric 3-D operator and of 2-D Poisson, row-scaled
    U = D_U (I + U_s): ||U_s||_2 <= ||U_s||_F <= sqrt(n (p - 1)) when the entries of U_s are at most 1
    (Theorem 1); 1/sqrt(rank) <= ||U_s||_2 when ||U_s||_2 < 1 < ||U_s||_F (Theorem 2); dep(I + U_s),
    which equals ||U_s||_F, is within the bounds of Theorems 3 and 4; Ruiz scaling lowers dep(U) of
    these badly row-scaled factors."""
    from oracle.nonnormal import factor_diagnostics, henrici_dep, split_factor

    O = oracle_lib
    for A in (convdiff3d(5, 3)[0], poisson2d(14)):
        F = O.ilut(A, droptol, lfil)
        d = factor_diagnostics(F)
        _, U = split_factor(F)
        Us = np.triu(U / np.diag(U)[:, None], 1)
        assert d["norm2_Us"] <= d["nu"] * (1 + 1e-12)
        if np.abs(Us).max() <= 1.0:
            assert d["nu"] <= d["th1_bound"]
        if d["norm2_Us"] < 1.0 < d["nu"]:
            assert 1.0 / np.sqrt(np.linalg.matrix_rank(Us)) <= d["norm2_Us"]
        dep1 = henrici_dep(np.eye(F.n) + Us)
        assert dep1 == pytest.approx(d["nu"], rel=1e-10)
        assert dep1 <= d["th3_bound"] and dep1 <= d["th4_bound"] * (1 + 1e-12)
        assert d["max_row_upper"] <= lfil + 1
    # a factor with rows of very different scale: Ruiz brings dep(U) down by orders of magnitude
    A = convdiff3d(5, 3)[0]
    w = np.exp(np.random.default_rng(0).uniform(-5, 5, A.n))
    As = CSR.from_dense(A.to_dense() * w[:, None])
    d = factor_diagnostics(O.ilut(As, 1e-2, 5))
    assert d["dep_U_ruiz"] < 1e-2 * d["dep_U"]


def test_ruiz_jacobi_equals_row_scaled_jacobi(oracle_lib):
    """Algorithm 2 with Ruiz scaling U~ = D_r U D_c, the transforms y~ = D_r y and v = D_c v~ (the ones that
    make U~ v~ = y~ equivalent to U v = y) and D = diag(U~)^{-1}: since diagonal scalings commute,
    D_c D D_r = D_U^{-1}, so every Jacobi iterate equals the row-scaled one (the smoother's form). With the
    transforms as printed (D_r^{-1} y, D_c^{-1} v~) the iteration does not solve U v = y."""
    from oracle.nonnormal import ruiz, split_factor

    O = oracle_lib
    A = convdiff3d(4, 3)[0]
    _, U = split_factor(O.ilut(A, 1e-2, 5))
    n = A.n
    dr, dc, _ = ruiz(U, 1e-12, 50)
    Ut = dr[:, None] * U * dc[None, :]
    D = 1.0 / np.diag(Ut)
    y = np.random.default_rng(8).standard_normal(n)
    v, vt, vp = np.zeros(n), np.zeros(n), np.zeros(n)
    yt, yp = dr * y, y / dr
    for _ in range(60):
        v = v + (y - U @ v) / np.diag(U)
        vt = vt + D * (yt - Ut @ vt)
        vp = vp + D * (yp - Ut @ vp)
        np.testing.assert_allclose(dc * vt, v, rtol=1e-11, atol=1e-13 * np.abs(v).max())
    assert np.linalg.norm(y - U @ v) <= 1e-12 * np.linalg.norm(y)
    assert np.linalg.norm(y - U @ (vp / dc)) > 1e-3 * np.linalg.norm(y)


def test_jacobi_triangular_residuals(oracle_lib):
    """Table 2's residuals: one iteration gives y = b and v = D_U^{-1} y, so the residuals are
    ||L_s b|| / ||b|| and ||strict(U) v|| / ||y||; at the dependency depth both solves are exact."""
    from oracle.nonnormal import jacobi_tri_residuals, split_factor

    O = oracle_lib
    A = poisson2d(9)
    F = O.ilut(A, 1e-3, 4)
    L, U = split_factor(F)
    b = np.random.default_rng(2).standard_normal(A.n)
    rl, ru = jacobi_tri_residuals(F, b, 1)
    assert rl == pytest.approx(np.linalg.norm((L - np.eye(A.n)) @ b) / np.linalg.norm(b), rel=1e-13)
    v = b / np.diag(U)
    assert ru == pytest.approx(np.linalg.norm(np.triu(U, 1) @ v) / np.linalg.norm(b), rel=1e-13)
    rl, ru = jacobi_tri_residuals(F, b, A.n)
    assert rl <= 1e-14 and ru <= 1e-13


def test_us_power_sequence_closed_form():
    """Section 5.3.2's power sequence on U = upper bidiagonal with (U_s)_{i,i+1} = a for every i: U_s = a J
    with J the shift, so U_s^p = a^p J^p has n - p entries, all a^p, and 2-norm |a|^p; it vanishes at p = n.
    The diagonal varies over powers of two, so the scaled superdiagonal is exactly a = -3/4."""
    from oracle.nonnormal import us_power_sequence

    n, a = 12, -0.75
    d = np.array([2.0 ** (i % 3) for i in range(n)])
    U = np.diag(d) + np.diag(a * d[:-1], 1)
    seq = us_power_sequence(CSR.from_dense(U), n + 2)
    for p in range(1, n + 3):
        expect = abs(a) ** p if p < n else 0.0
        assert seq["max_abs"][p - 1] == expect
        assert seq["norm2"][p - 1] == pytest.approx(expect, rel=1e-14, abs=0.0)
        assert seq["nnz"][p - 1] == max(n - p, 0)


def test_us_power_sequence_nilpotency_and_bounds(oracle_lib):
    """On ILUT factors of a 3-D Poisson matrix (an M-matrix, so every entry of U_s is <= 0 and the entries
    of U_s^p share the sign (-1)^p: no cancellation), nnz(U_s^p) equals the number of index pairs joined by
    a path of exactly p edges in U_s's graph (brute force on the pattern), the powers vanish exactly one
    step past the longest chain, and max |(U_s^p)_ij| <= ||U_s^p||_2 <= ||U_s||_2^p."""
    from oracle.nonnormal import split_factor, us_power_sequence

    O = oracle_lib
    A = poisson3d(4)
    for droptol, lfil in ((1e-2, 5), (1e-3, 20)):
        F = O.ilut(A, droptol, lfil)
        _, U = split_factor(F)
        Us = np.triu(U / np.diag(U)[:, None], 1)
        assert (Us <= 0).all()
        n = A.n
        depth = np.zeros(n, dtype=int)  # edges of the longest chain starting at i
        for i in range(n - 1, -1, -1):
            js = np.nonzero(Us[i])[0]
            depth[i] = 1 + depth[js].max() if len(js) else 0
        chain = int(depth.max())
        seq = us_power_sequence(F, chain + 2)
        B = (Us != 0).astype(np.int64)
        R = np.eye(n, dtype=np.int64)
        for p in range(1, chain + 3):
            R = np.minimum(R @ B, 1)  # pairs joined by a path of exactly p edges
            assert seq["nnz"][p - 1] == int(R.sum()), (droptol, p)
        assert (seq["nnz"][:chain] > 0).all() and seq["nnz"][chain] == 0 and seq["nnz"][chain + 1] == 0
        s1 = seq["norm2"][0]
        for p in range(1, chain + 1):
            assert seq["max_abs"][p - 1] <= seq["norm2"][p - 1] * (1 + 1e-12)
            assert seq["norm2"][p - 1] <= s1 ** p * (1 + 1e-12)


# ------------------------------------------------------------- aggressive (A-1) coarsening, Section 5.1
def _dist2_cc_graph(srp, sci, cf):
    """Brute force: for each first-pass C point, the C points reachable by one or two strong connections."""
    S = [set(sci[srp[i]:srp[i + 1]]) for i in range(len(srp) - 1)]
    C = np.nonzero(cf == 1)[0]
    pos = {c: q for q, c in enumerate(C)}
    G = []
    for i in C:
        reach = set(S[i])
        for k in S[i]:
            reach |= S[k]
        G.append({pos[j] for j in reach if j in pos and j != i})
    return C, G


@pytest.mark.parametrize("maker", [lambda: poisson2d(24), lambda: poisson3d(12), lambda: convdiff3d(12, 3)[0],
                                   lambda: varcoef3d(12, 1.0, 2, 100.0)[0]])
def test_aggressive_coarsening_structure(oracle_lib, maker):
    """A-1 aggressive coarsening on the finest level: the final C points are a subset of the first
    pass's C points, chosen by an RS first pass on the distance-two strength among them (every C point
    that is dropped has a kept point among its one- or two-step strong connections); P = P_1 P_2 keeps
    the identity rows of the kept points; the coarse operator is the Galerkin product P^T A P (dense
    check); and the hierarchy has fewer coarse unknowns and a lower operator complexity than standard
    coarsening."""
    O = oracle_lib
    A = maker()
    theta = 0.25
    cf1 = O.coarsen(A, theta)
    srp, sci = O.strength(A, theta)
    C1, G = _dist2_cc_graph(srp, sci, cf1)
    H = O.Hierarchy(A, theta=theta, agg_levels=1)
    H0 = O.Hierarchy(A, theta=theta)
    lv0, lv1 = H.level(0), H.level(1)
    cf = lv0.cf
    assert np.all(cf[cf1 == 0] == 0)  # C_2 within C_1
    keep = cf[C1] == 1
    assert 0 < keep.sum() < len(C1)
    for q in np.nonzero(~keep)[0]:
        if G[q] or any(q in G[r] for r in range(len(G))):
            assert any(keep[r] for r in G[q]), q
    P = lv0.P.toarray()
    cidx = np.cumsum(cf) - 1
    for i in np.nonzero(cf == 1)[0]:
        row = np.zeros(P.shape[1])
        row[cidx[i]] = 1.0
        np.testing.assert_array_equal(P[i], row)
    Ad = A.to_dense()
    Ac = lv1.A.to_dense()
    np.testing.assert_allclose(Ac, P.T @ Ad @ P, atol=1e-12 * np.abs(Ac).max())
    nnz = [H.level(l).A.nnz for l in range(H.levels)]
    nnz0 = [H0.level(l).A.nnz for l in range(H0.levels)]
    assert lv1.A.n < H0.level(1).A.n and sum(nnz) < sum(nnz0)


def test_aggressive_coarsening_solves(oracle_lib):
    """With aggressive coarsening on the first two levels (as in Section 6.1) the preconditioned solve
    still reaches the true relative residual; agg_levels < 0 is rejected."""
    O = oracle_lib
    for name, N, sm, t in (("c1", None, 0, 2), ("c2", 16, 1, 3), ("c3", 16, 0, 2)):
        A, b, _ = __import__("workloads").config_system(name, N)
        r = O.Hierarchy(A, agg_levels=2).solve(b, smoother=sm, t=t)
        assert r["status"] == 0 and np.linalg.norm(b - A.to_dense() @ r["x"]) <= 1e-8 * np.linalg.norm(b)
    with pytest.raises(O.OracleFailure):
        O.Hierarchy(poisson2d(10), agg_levels=-1)


# -------------------------------------------------- PMIS and BAMG direct interpolation (Section 5.1)
def test_splitmix64_reference_outputs(oracle_lib):
    """The generator behind PMIS's random weights is SplitMix64 as published: its first four outputs from
    state 0 (tests/golden/splitmix64_state0.json); the draw of point i is output i + 1 scaled to [0, 1)."""
    g = json.load(open(os.path.join(GOLD, "splitmix64_state0.json")))
    O = oracle_lib
    assert [O.splitmix64(g["state"], k) for k in range(1, 5)] == [int(h, 16) for h in g["outputs_hex"]]
    for seed, i in ((0, 0), (0, 3), (5, 1000), (2 ** 63 + 11, 7)):
        u = O.uniform01(seed, i)
        assert 0.0 <= u < 1.0 and u == (O.splitmix64(seed, i + 1) >> 11) / 2.0 ** 53


def _strong_lists(O, A, theta=0.25):
    srp, sci = O.strength(A, theta)
    S = [list(sci[srp[i]:srp[i + 1]]) for i in range(A.n)]
    ST = [[] for _ in range(A.n)]
    for i, row in enumerate(S):
        for j in row:
            ST[j].append(i)
    return S, ST


@pytest.mark.parametrize("maker", [lambda: poisson2d(20), lambda: poisson3d(9), lambda: convdiff3d(9, 3)[0],
                                   lambda: varcoef3d(9, 1.0, 2, 100.0)[0], lambda: random_csr(200, 6, 4)])
@pytest.mark.parametrize("seed", [0, 12345])
def test_pmis_splitting_properties(oracle_lib, maker, seed):
    """PMIS (Section 5.1) on the finest level, checked against its definition with the weights recomputed
    from the pinned generator: a point that influences no other point is F; every other F point strongly
    depends on a C point; and a C point that strongly depends on another C point has the larger weight
    (it was chosen while the other was still undecided and adjacent)."""
    O = oracle_lib
    A = maker()
    S, ST = _strong_lists(O, A)
    H = O.Hierarchy(A, coarsen=O.COARSEN_PMIS, seed=seed, max_levels=2, max_coarse=1)
    cf = H.level(0).cf
    w = np.array([len(ST[i]) + O.uniform01(seed, i) for i in range(A.n)])
    for i in range(A.n):
        if not ST[i]:
            assert cf[i] == 0, i
        elif cf[i] == 0:
            assert any(cf[j] == 1 for j in S[i]), i
        else:
            for j in S[i]:
                if cf[j] == 1:
                    assert w[i] > w[j] or (w[i] == w[j] and i < j), (i, j)
    assert 0 < cf.sum() < A.n


@pytest.mark.parametrize("maker", [lambda: poisson2d(16), lambda: convdiff3d(8, 3)[0], lambda: varcoef3d(8, 1.0, 2, 100.0)[0]])
def test_bamg_direct_interpolation(oracle_lib, maker):
    """BAMG direct interpolation (Section 5.1): C rows are identity rows; an F row interpolates from
    exactly its strong C neighbours (none: empty row); on zero-row-sum rows the weights solve the local
    problem min || a~_ii w + a_{i,C} || subject to w^T 1 = 1 (a~_ii: the diagonal with the weak
    neighbours added), computed here from its KKT system, and therefore interpolate constants."""
    O = oracle_lib
    A = maker()
    S, _ = _strong_lists(O, A)
    H = O.Hierarchy(A, coarsen=O.COARSEN_PMIS, seed=3, max_levels=2, max_coarse=1)
    lv = H.level(0)
    cf, P = lv.cf, lv.P.tocsr()
    cidx = np.cumsum(cf) - 1
    Ad = A.to_dense()
    checked = 0
    for i in range(A.n):
        row = P.getrow(i)
        if cf[i] == 1:
            assert list(row.indices) == [cidx[i]] and list(row.data) == [1.0]
            continue
        Ci = [j for j in S[i] if cf[j] == 1]
        assert sorted(row.indices) == sorted(cidx[j] for j in Ci)
        if not Ci or abs(Ad[i].sum()) > 1e-12 * np.abs(Ad[i]).max():
            continue
        weak = [k for k in np.nonzero(Ad[i])[0] if k != i and k not in S[i]]
        at = Ad[i, i] + Ad[i, weak].sum()
        m = len(Ci)
        K = np.zeros((m + 1, m + 1))
        K[:m, :m] = 2 * at * at * np.eye(m)
        K[:m, m] = K[m, :m] = 1.0
        rhs = np.concatenate([-2 * at * Ad[i, Ci], [1.0]])
        wk = np.linalg.solve(K, rhs)[:m]
        got = np.array([P[i, cidx[j]] for j in Ci])
        np.testing.assert_allclose(got, wk, rtol=1e-12, atol=1e-14)
        assert got.sum() == pytest.approx(1.0, rel=1e-13)
        checked += 1
    assert checked > 0


def test_pmis_hierarchy_solves_and_seeds(oracle_lib):
    """The PMIS + BAMG direct hierarchy is deterministic for a seed, changes with it, and as a
    preconditioner reaches the true relative residual; it does not combine with aggressive coarsening."""
    O = oracle_lib
    A, b, _ = __import__("workloads").config_system("c2", 16)
    H1, H2 = O.Hierarchy(A, coarsen=O.COARSEN_PMIS, seed=1), O.Hierarchy(A, coarsen=O.COARSEN_PMIS, seed=1)
    H3 = O.Hierarchy(A, coarsen=O.COARSEN_PMIS, seed=2)
    assert np.array_equal(H1.level(0).cf, H2.level(0).cf) and not np.array_equal(H1.level(0).cf, H3.level(0).cf)
    for sm, t in ((0, 2), (1, 3)):
        r = H1.solve(b, smoother=sm, t=t)
        assert r["status"] == 0 and np.linalg.norm(b - A.to_dense() @ r["x"]) <= 1e-8 * np.linalg.norm(b)
    with pytest.raises(O.OracleFailure):
        O.Hierarchy(A, coarsen=O.COARSEN_PMIS, agg_levels=1)
    with pytest.raises(O.OracleFailure):
        O.Hierarchy(A, coarsen=2)
