"""The seeded input generators against plain per-cell loops written from their definitions (CPU).

The variable-coefficient generator computes every interior face once for both of its cells; this checks,
bit for bit on small grids (stretched and not), that it equals the definition cell by cell: faces in the
order -x, +x, -y, +y, -z, +z, T = area / (h_c/(2k_c) + h_c'/(2k_c')), a boundary face area / (h_c/(2k_c)),
a_cc the running sum of the row's T from 0, a_cc' = -T, columns ascending.
"""
import numpy as np
import pytest

from workloads import serve_stream, varcoef3d
from workloads.stencils import stretched_spacing


def varcoef_by_cells(N, sigma, seed, stretch):
    rng = np.random.default_rng(seed)
    n = N ** 3
    kappa = np.exp(sigma * rng.standard_normal(n))
    b = rng.standard_normal(n)
    h = [np.full(N, 1.0 / N), np.full(N, 1.0 / N), stretched_spacing(N, stretch)]
    stride = [1, N, N * N]
    rp, ci, vals = [0], [], []
    for c in range(n):
        coord = [c % N, (c // N) % N, c // (N * N)]
        w = [h[a][coord[a]] for a in range(3)]
        diag = 0.0
        entries = {}
        for a in range(3):
            area = float(w[(a + 1) % 3] * w[(a + 2) % 3])
            half_own = float(w[a] / (2.0 * kappa[c]))
            for s in (-1, 1):
                q = coord[a] + s
                if 0 <= q < N:
                    o = c + s * stride[a]
                    half_other = float(h[a][q] / (2.0 * kappa[o]))
                    t = area / (half_own + half_other)
                    entries[o] = -t
                else:
                    t = area / half_own
                diag += t
        entries[c] = diag
        for col in sorted(entries):
            ci.append(col)
            vals.append(entries[col])
        rp.append(len(ci))
    return np.array(rp), np.array(ci), np.array(vals), b


@pytest.mark.parametrize("N,stretch", [(1, 1.0), (2, 1.0), (5, 1.0), (6, 100.0), (9, 3.0)])
def test_varcoef_matches_cell_by_cell_definition(N, stretch):
    A, b = varcoef3d(N, 0.7, 40 + N, stretch)
    rp, ci, v, b2 = varcoef_by_cells(N, 0.7, 40 + N, stretch)
    assert np.array_equal(A.rowptr, rp) and np.array_equal(A.colind, ci)
    assert np.array_equal(A.vals, v) and np.array_equal(b, b2)


def test_varcoef_is_thread_safe_and_deterministic():
    from concurrent.futures import ThreadPoolExecutor

    sizes = [7, 9, 7, 11, 9, 7, 13, 11]
    with ThreadPoolExecutor(4) as ex:
        got = list(ex.map(lambda j: varcoef3d(sizes[j], 0.5, 1000 + j), range(len(sizes))))
    for j, (A, b) in enumerate(got):
        B, c = varcoef3d(sizes[j], 0.5, 1000 + j)
        assert np.array_equal(A.vals, B.vals) and np.array_equal(A.colind, B.colind) and np.array_equal(b, c)


def test_serve_stream_shape():
    """2000 Poisson arrivals at 50/s (mean gap 20 ms) with n log-uniform in [32, 160]."""
    r = serve_stream(2000, seed=5)
    t = np.array([q["arrival_s"] for q in r])
    N = np.array([q["N"] for q in r])
    assert len(r) == 2000 and np.all(np.diff(t) > 0)
    assert 0.018 < t[-1] / 2000 < 0.022
    assert N.min() >= 32 and N.max() <= 160
    assert [q["seed"] for q in r[:3]] == [1000, 1001, 1002]
