"""Non-normality diagnostics of incomplete triangular factors (Sections 5.3.1 to 5.3.4: Henrici's departure
from normality, 5.3.1; the powers of U_s that the Neumann series sums, 5.3.2; the Jacobi triangular-solve
residuals of Table 2, 5.3.3; Theorems 1 to 4 and Ruiz scaling, 5.3.4).

Plain dense numpy definitions for small matrices. Test infrastructure, like the rest of the oracle: only
the tests and the benchmark's CPU leg import it.

F is a factor CSR holding L \\ U (strict lower part = L_s of the unit-diagonal L; diagonal and strict
upper part = U), as returned by oracle.ilut or built from oracle.ilu0.
"""
from __future__ import annotations

import numpy as np


def split_factor(F):
    """Dense (L, U) from a factor CSR: L = I + L_s, U upper triangular with its diagonal."""
    d = F.to_dense()
    return np.tril(d, -1) + np.eye(F.n), np.triu(d)


def henrici_dep(T):
    """Henrici's departure from normality: dep(T)^2 = ||T||_F^2 - sum_i |lambda_i(T)|^2 (clamped at 0)."""
    lam = np.linalg.eigvals(T)
    return float(np.sqrt(max(np.linalg.norm(T, "fro") ** 2 - np.sum(np.abs(lam) ** 2), 0.0)))


def ruiz(M, tol=1e-8, max_iters=20):
    """Ruiz's simultaneous row and column equilibration in the infinity norm: with r_i and c_j the largest
    magnitudes in row i and column j of the current scaled matrix, scale rows by 1/sqrt(r_i) and columns
    by 1/sqrt(c_j) together, until every r_i and c_j is within tol of 1 or max_iters iterations have run.
    Returns (d_r, d_c, iterations) with the scaled matrix diag(d_r) M diag(d_c)."""
    M = np.abs(np.asarray(M, dtype=np.float64))
    n, m = M.shape
    dr, dc = np.ones(n), np.ones(m)
    it = 0
    while True:
        S = dr[:, None] * M * dc[None, :]
        r, c = S.max(axis=1), S.max(axis=0)
        if max(np.abs(1.0 - r).max(), np.abs(1.0 - c).max()) <= tol or it >= max_iters:
            return dr, dc, it
        dr = dr / np.sqrt(r)
        dc = dc / np.sqrt(c)
        it += 1


def factor_diagnostics(F, ruiz_tol=1e-8, ruiz_max_iters=20):
    """The quantities of Section 5.3.4 for the factor F, by their definitions:
    dep_L = dep(L), dep_U = dep(U) (unscaled), nu = ||U_s||_F and norm2_Us = ||U_s||_2 for the row-scaled
    U = D_U (I + U_s); p = the most stored entries in a row of U (diagonal included); the bounds of
    Theorem 1 (sqrt(n (p - 1))), Theorem 3 (sqrt((2 sqrt(n) + nu) nu)) and Theorem 4 (sqrt(n) (1 + delta),
    delta = max_i max(0, sum_j |(U_s)_ij| - 1)); dep(D_r U D_c) after Ruiz scaling of U."""
    n = F.n
    L, U = split_factor(F)
    du = np.diag(U)
    Us = np.triu(U / du[:, None], 1)
    p = int(max(np.count_nonzero(U[i]) for i in range(n)))
    nu = float(np.linalg.norm(Us, "fro"))
    delta = float(max(0.0, (np.abs(Us).sum(axis=1) - 1.0).max()))
    dr, dc, it = ruiz(U, ruiz_tol, ruiz_max_iters)
    Ur = dr[:, None] * U * dc[None, :]
    return {
        "n": n,
        "max_row_upper": p,
        "dep_L": henrici_dep(L),
        "dep_U": henrici_dep(U),
        "nu": nu,
        "norm2_Us": float(np.linalg.norm(Us, 2)),
        "th1_bound": float(np.sqrt(n * (p - 1))),
        "th3_bound": float(np.sqrt((2.0 * np.sqrt(n) + nu) * nu)),
        "delta": delta,
        "th4_bound": float(np.sqrt(n) * (1.0 + delta)),
        "dep_U_ruiz": henrici_dep(Ur),
        "ruiz_iters": it,
    }


def jacobi_tri_residuals(F, b, iters):
    """Table 2's measure: `iters` Jacobi iterations from zero for L y = b (y <- y + (b - L y)), then for
    U v = y with the row scaling D = diag(U)^{-1} (v <- v + D (y - U v)); returns
    (||b - L y|| / ||b||, ||y - U v|| / ||y||)."""
    L, U = split_factor(F)
    y = np.zeros(F.n)
    for _ in range(iters):
        y = y + (b - L @ y)
    v = np.zeros(F.n)
    d = 1.0 / np.diag(U)
    for _ in range(iters):
        v = v + d * (y - U @ v)
    return (float(np.linalg.norm(b - L @ y) / np.linalg.norm(b)),
            float(np.linalg.norm(y - U @ v) / np.linalg.norm(y)))


def us_power_sequence(F, pmax):
    """The sequence that Section 5.3.2 plots for a factor (its figure of max |(U_s^p)_ij|, ||U_s^p||_2 and
    nnz(U_s^p) against p): for p = 1..pmax, the largest magnitude, the 2-norm and the number of nonzero
    entries of the p-th power of U_s = D_U^{-1} U - I, the strictly upper triangular part of the row-scaled
    U. U_s is nilpotent, so the powers vanish once p exceeds the longest chain of its graph; the Neumann
    form of the U solve sums the terms (-U_s)^j, and these numbers say how fast they decay."""
    _, U = split_factor(F)
    Us = np.triu(U / np.diag(U)[:, None], 1)
    P = np.eye(F.n)
    max_abs, norm2, nnz = [], [], []
    for _ in range(pmax):
        P = P @ Us
        max_abs.append(float(np.abs(P).max()) if P.size else 0.0)
        norm2.append(float(np.linalg.norm(P, 2)) if P.size else 0.0)
        nnz.append(int(np.count_nonzero(P)))
    return {"max_abs": np.array(max_abs), "norm2": np.array(norm2), "nnz": np.array(nnz, dtype=np.int64)}
