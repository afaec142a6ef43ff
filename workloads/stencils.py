"""Seeded generators for the pressure-type systems the solver is measured on.

The paper measures on Nalu-Wind and PeleLM pressure matrices (Section 6), which are not available here;
these generators stand in for them with the same shapes: 5/7-point pressure Poisson stencils, a
variable-coefficient finite-volume operator with a stretched mesh, and a mildly nonsymmetric upwind
convection-diffusion operator (the Nalu-Wind systems are slightly nonsymmetric, Section 5.3.3).

Conventions, identical for every consumer:
  * unknowns are numbered lexicographically, x fastest: idx = x + nx*(y + ny*z);
  * Dirichlet boundaries are eliminated, so the stencil only couples interior unknowns;
  * CSR is 0-based with int32 row pointers and column indices, columns ascending, diagonal present,
    values float64;
  * every random draw comes from numpy.random.default_rng(seed) (PCG64) in a fixed order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int32[n+1]
    colind: np.ndarray  # int32[nnz]
    vals: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        for i in range(self.n):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            d[i, self.colind[s:e]] = self.vals[s:e]
        return d

    @staticmethod
    def from_scipy(m) -> "CSR":
        m = m.tocsr()
        m.sort_indices()
        return CSR(
            m.shape[0],
            np.ascontiguousarray(m.indptr, dtype=np.int32),
            np.ascontiguousarray(m.indices, dtype=np.int32),
            np.ascontiguousarray(m.data, dtype=np.float64),
        )

    @staticmethod
    def from_dense(d: np.ndarray) -> "CSR":
        n = d.shape[0]
        rp = [0]
        ci: list[int] = []
        v: list[float] = []
        for i in range(n):
            for j in range(n):
                if d[i, j] != 0.0 or i == j:
                    ci.append(j)
                    v.append(float(d[i, j]))
            rp.append(len(ci))
        return CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, np.float64))


def _assemble(dims, diag, nbr):
    """Build CSR from per-unknown coefficients.

    dims: (nx, ny, nz); diag: float64[n]; nbr: list of (axis, step, coeff float64[n]) giving the
    coefficient that row p places on unknown p + step*e_axis (dropped where that unknown is outside
    the grid, i.e. a Dirichlet boundary).
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    coord = [idx % nx, (idx // nx) % ny, idx // (nx * ny)]
    stride = [1, nx, nx * ny]
    extent = [nx, ny, nz]
    entries = []  # (offset, col array, val array, mask)
    for axis, step, coeff in nbr:
        c = coord[axis] + step
        mask = (c >= 0) & (c < extent[axis])
        off = step * stride[axis]
        entries.append((off, idx + off, coeff, mask))
    entries.append((0, idx, diag, np.ones(n, bool)))
    entries.sort(key=lambda e: e[0])  # ascending column offset == ascending column index per row
    cols = np.stack([e[1] for e in entries], axis=1)
    vals = np.stack([np.broadcast_to(e[2], (n,)) for e in entries], axis=1)
    mask = np.stack([e[3] for e in entries], axis=1)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    return CSR(
        n,
        rowptr.astype(np.int32),
        cols[mask].astype(np.int32),
        np.ascontiguousarray(vals[mask], dtype=np.float64),
    )


def tridiag1d(n: int) -> CSR:
    """tridiag(-1, 2, -1) on n interior points."""
    one = np.ones(n)
    return _assemble((n, 1, 1), 2.0 * one, [(0, -1, -one), (0, 1, -one)])


def poisson2d(N: int) -> CSR:
    """5-point Laplacian on an N x N interior grid: a_pp = 4, a_pq = -1."""
    one = np.ones(N * N)
    nbr = [(0, -1, -one), (0, 1, -one), (1, -1, -one), (1, 1, -one)]
    return _assemble((N, N, 1), 4.0 * one, nbr)


def poisson3d(N: int) -> CSR:
    """7-point Laplacian on an N^3 interior grid: a_pp = 6, a_pq = -1."""
    one = np.ones(N ** 3)
    nbr = [(a, s, -one) for a in range(3) for s in (-1, 1)]
    return _assemble((N, N, N), 6.0 * one, nbr)


def stretched_spacing(N: int, ratio: float) -> np.ndarray:
    """Geometric spacings h_k = h0 q^k, k < N, with h_{N-1}/h_0 = ratio and sum 1."""
    if ratio == 1.0:
        return np.full(N, 1.0 / N)
    q = ratio ** (1.0 / (N - 1))
    h = q ** np.arange(N, dtype=np.float64)
    return h / h.sum()


def varcoef3d(N: int, sigma: float, seed: int, stretch: float = 1.0):
    """Cell-centred finite volumes for -div(k grad p) on the unit cube, N^3 cells, Dirichlet p = 0.

    k = exp(sigma * xi) per cell with xi ~ N(0, 1); hx = hy = 1/N; z spacing geometric with
    hz_max/hz_min = stretch. Face transmissibility T = area / (h_c/(2k_c) + h_c'/(2k_c')); a boundary
    face uses area / (h_c/(2k_c)). Row c: a_cc = sum of its face T (faces in the order -x, +x, -y, +y,
    -z, +z), a_cc' = -T. SPD M-matrix. Returns (A, b) with b ~ N(0, 1) drawn after k from the same
    generator.

    Each interior face is computed once: both of its cells see the same area and the same two half-cell
    resistances, whose sum does not depend on their order. The sparsity structure of an N^3 grid is
    shared by every system of that size (cached).
    """
    rng = np.random.default_rng(seed)
    n = N ** 3
    kappa = np.exp(sigma * rng.standard_normal(n))
    b = rng.standard_normal(n)
    hx = np.full(N, 1.0 / N)
    hz = stretched_spacing(N, stretch)
    two_k = 2.0 * kappa.reshape(N, N, N)  # [z, y, x]
    # width of every cell along grid axis a (x, y, z), broadcast over [z, y, x]
    width = [np.broadcast_to(hx[None, None, :], (N, N, N)), np.broadcast_to(hx[None, :, None], (N, N, N)),
             np.broadcast_to(hz[:, None, None], (N, N, N))]
    dim = [2, 1, 0]  # array dimension of grid axis a
    diag = np.zeros((N, N, N))
    coef = {}
    for a in range(3):
        area = width[(a + 1) % 3] * width[(a + 2) % 3]
        half = width[a] / two_k
        lo, hi, first, last = ([slice(None)] * 3 for _ in range(4))
        lo[dim[a]], hi[dim[a]] = slice(0, N - 1), slice(1, N)
        first[dim[a]], last[dim[a]] = slice(0, 1), slice(N - 1, N)
        lo, hi, first, last = tuple(lo), tuple(hi), tuple(first), tuple(last)
        face = area[lo] / (half[lo] + half[hi])  # between cell i and cell i + 1 along a
        minus, plus = np.empty((N, N, N)), np.empty((N, N, N))
        minus[first] = area[first] / half[first]
        minus[hi] = face
        plus[last] = area[last] / half[last]
        plus[lo] = face
        diag += minus
        diag += plus
        coef[(a, -1)], coef[(a, 1)] = minus, plus
    rowptr, colind, keep = _grid7_structure(N)
    slots = [coef[(2, -1)], coef[(1, -1)], coef[(0, -1)], None, coef[(0, 1)], coef[(1, 1)], coef[(2, 1)]]
    vals = np.empty((n, 7))
    for j, c in enumerate(slots):
        if c is None:
            vals[:, j] = diag.ravel()
        else:
            np.negative(c.ravel(), out=vals[:, j])
    return CSR(n, rowptr, colind, np.ascontiguousarray(vals[keep])), b


_GRID7_CACHE: dict = {}
_GRID7_LOCK = __import__("threading").Lock()


def _grid7_structure(N: int):
    """Row pointers, column indices and the entry mask (n x 7, slots in ascending column order
    -N^2, -N, -1, 0, +1, +N, +N^2) of the 7-point stencil on an N^3 grid with Dirichlet boundaries
    eliminated. The few most recent sizes are kept."""
    with _GRID7_LOCK:
        hit = _GRID7_CACHE.get(N)
    if hit is not None:
        return hit
    n = N ** 3
    z, y, x = np.ogrid[0:N, 0:N, 0:N]
    conds = [z > 0, y > 0, x > 0, np.ones((1, 1, 1), bool), x < N - 1, y < N - 1, z < N - 1]
    keep = np.empty((n, 7), bool)
    for j, c in enumerate(conds):
        keep[:, j] = np.broadcast_to(c, (N, N, N)).ravel()
    cols = np.arange(n, dtype=np.int32)[:, None] + np.array([-N * N, -N, -1, 0, 1, N, N * N], np.int32)[None, :]
    colind = np.ascontiguousarray(cols[keep])
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(keep.sum(axis=1), out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    out = (rowptr.astype(np.int32), colind, keep)
    with _GRID7_LOCK:
        if len(_GRID7_CACHE) >= 4:
            _GRID7_CACHE.pop(next(iter(_GRID7_CACHE)))
        _GRID7_CACHE[N] = out
    return out


def convdiff3d(N: int, seed: int, peclet: float = 10.0):
    """-Lap(u) + w.grad(u) on an N^3 interior grid, h = 1/(N+1), first-order upwind, scaled by h^2.

    w = peclet * U(-1, 1) per node and component. a_pp = 6 + h*sum_d |w_d|; along axis d the upwind
    neighbour gets -1 - h|w_d| and the downwind one -1. Returns (A, b, perm) where b ~ N(0, 1) and perm
    is a random permutation of the unknowns, all drawn in that order from default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    n = N ** 3
    h = 1.0 / (N + 1)
    w = peclet * rng.uniform(-1.0, 1.0, (n, 3))
    b = rng.standard_normal(n)
    perm = rng.permutation(n)
    diag = 6.0 + h * np.abs(w).sum(axis=1)
    nbr = []
    for a in range(3):
        wa = w[:, a]
        up_minus = wa > 0  # flow in +e_a: upwind neighbour is p - e_a
        up_plus = wa < 0
        nbr.append((a, -1, np.where(up_minus, -1.0 - h * np.abs(wa), -1.0)))
        nbr.append((a, 1, np.where(up_plus, -1.0 - h * np.abs(wa), -1.0)))
    return _assemble((N, N, N), diag, nbr), b, perm


def permute_symmetric(A: CSR, perm: np.ndarray) -> CSR:
    """B = A[perm][:, perm], i.e. B_ij = A_{perm[i], perm[j]} (a symmetric relabelling)."""
    m = A.to_scipy()[perm][:, perm]
    return CSR.from_scipy(m)


def rcm_permutation(A: CSR) -> np.ndarray:
    """Reverse Cuthill-McKee ordering of a structurally symmetric matrix (scipy)."""
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    return np.asarray(reverse_cuthill_mckee(A.to_scipy(), symmetric_mode=True), dtype=np.int64)


def random_csr(n: int, per_row: int, seed: int, symmetric: bool = False, dominance: float = 1.5) -> CSR:
    """Random sparse matrix with sorted columns and a dominant positive diagonal (test inputs)."""
    rng = np.random.default_rng(seed)
    d = np.zeros((n, n))
    for i in range(n):
        cols = rng.choice(n, size=min(per_row, n), replace=False)
        d[i, cols] = rng.uniform(-1.0, 0.2, cols.size)
    if symmetric:
        d = 0.5 * (d + d.T)
    np.fill_diagonal(d, 0.0)
    np.fill_diagonal(d, dominance * np.abs(d).sum(axis=1) + 1.0)
    return CSR.from_dense(d)


# ----------------------------------------------------------------------------------------------
# The five measured configurations.

def config_system(name: str, N: int | None = None):
    """Return (A, b, meta) for a named configuration; N overrides the grid size for small tests.

    c1: 2-D Poisson 32^2, b ~ U(-1, 1) seed 0.
    c2: 3-D Poisson 128^3, b ~ N(0, 1) seed 1.
    c3: -div(k grad p), 192^3, k lognormal sigma = 1 seed 2, z stretched 1:100.
    c4n / c4r / c4rcm: upwind convection-diffusion 128^3 seed 3 in natural, random-relabelled and
        RCM-of-random orderings.
    """
    if name == "c1":
        N = N or 32
        A = poisson2d(N)
        b = np.random.default_rng(0).uniform(-1.0, 1.0, A.n)
    elif name == "c2":
        N = N or 128
        A = poisson3d(N)
        b = np.random.default_rng(1).standard_normal(A.n)
    elif name == "c3":
        N = N or 192
        A, b = varcoef3d(N, 1.0, 2, stretch=100.0)
    elif name in ("c4n", "c4r", "c4rcm"):
        N = N or 128
        A, b, perm = convdiff3d(N, 3)
        if name != "c4n":
            A = permute_symmetric(A, perm)
            b = b[perm]
            if name == "c4rcm":
                q = rcm_permutation(A)
                A = permute_symmetric(A, q)
                b = b[q]
    else:
        raise ValueError(f"unknown configuration {name!r}")
    return A, np.ascontiguousarray(b, dtype=np.float64), {"name": name, "N": N}


def serve_stream(count: int = 2000, seed: int = 5, rate_hz: float = 50.0, nmin: int = 32, nmax: int = 160):
    """Request stream: Poisson arrivals at rate_hz and grid sizes n log-uniform in [nmin, nmax].

    Returns a list of dicts {arrival_s, N, seed}; request j's system is varcoef3d(N, 0.5, seed)
    with seed = 1000 + j and no stretch.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, count)
    sizes = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), count))).astype(int)
    t = np.cumsum(gaps)
    return [{"arrival_s": float(t[j]), "N": int(sizes[j]), "seed": 1000 + j} for j in range(count)]
