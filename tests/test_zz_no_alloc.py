"""The allocation-free solve entry point (namg_solve_noalloc) against namg_solve, through the C ABI.

namg_solve_noalloc runs namg_solve's kernels with the Krylov workspace in the library's static per-device
array. Two calls in a row on one device, the second on a smaller system (the array keeps the first call's
contents), must each give the same x bit for bit, the same iteration count and the same residuals as
namg_solve on the same hierarchy and inputs, and must leave the hierarchy's own device memory unchanged (no
workspace is allocated). A workspace larger than the static array, and the options that allocate on first
use, are refused with NAMG_E_INVALID before any work is issued.
"""
import numpy as np
import pytest

from workloads import config_system, poisson2d

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def namg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_14681_amd as m

    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _same_solve(a, b):
    assert a["status"] == b["status"]
    assert a["iters"] == b["iters"] and a["cycles"] == b["cycles"]
    assert a["relres_true"] == b["relres_true"] and a["relres_est"] == b["relres_est"]


def test_noalloc_matches_solve_two_calls_second_smaller(namg):
    # call 1: 3-D Poisson 24^3 (13 824 rows), FP32 preconditioner, hybrid ILU(0) t = 3, GMRES(30)
    A1, b1, _ = config_system("c2", 24)
    H1 = namg.Hierarchy(A1, device=0, precision=namg.FP32_PRECOND)
    p1 = dict(tol=1e-8, restart=30, smoother=namg.SMOOTH_ILU0, inner_terms=3)
    # call 2: 2-D Poisson 32^2 (1 024 rows), all FP64, polynomial GS t = 2, GMRES(20), x0 != 0
    A2, b2, _ = config_system("c1")
    H2 = namg.Hierarchy(A2, device=0)
    p2 = dict(tol=1e-10, restart=20, smoother=namg.SMOOTH_PGS, inner_terms=2)
    x02 = np.random.default_rng(7).uniform(-1, 1, A2.n)
    assert A2.n < A1.n

    bytes1, bytes2 = H1.info()["device_bytes"], H2.info()["device_bytes"]
    bt1, bt2 = dev(b1), dev(b2)
    xa1, xa2 = torch.zeros_like(bt1), dev(x02)
    print(f"[noalloc] call 1: n {A1.n} FP32 precond; call 2: n {A2.n} FP64", flush=True)
    s_a1 = H1.solve_noalloc(bt1, xa1, history=True, **p1)
    s_a2 = H2.solve_noalloc(bt2, xa2, history=True, **p2)
    xa1, xa2 = host(xa1), host(xa2)
    # no workspace was allocated for either hierarchy
    assert H1.info()["device_bytes"] == bytes1 and H2.info()["device_bytes"] == bytes2

    xr1, xr2 = torch.zeros_like(bt1), dev(x02)
    s_r1 = H1.solve(bt1, xr1, history=True, **p1)
    s_r2 = H2.solve(bt2, xr2, history=True, **p2)
    xr1, xr2 = host(xr1), host(xr2)
    assert H1.info()["device_bytes"] > bytes1  # namg_solve allocates its workspace on first use

    for sa, sr, xa, xr in ((s_a1, s_r1, xa1, xr1), (s_a2, s_r2, xa2, xr2)):
        print(f"[noalloc] iters {sa['iters']} relres {sa['relres_true']:.3e}; namg_solve iters {sr['iters']} "
              f"relres {sr['relres_true']:.3e}; max |x diff| {np.abs(xa - xr).max():.1e}", flush=True)
        assert sa["status"] == namg.OK and sa["relres_true"] <= 1e-8
        _same_solve(sa, sr)
        assert np.array_equal(sa["hist"], sr["hist"])
        assert np.array_equal(xa, xr)

    # again on the larger system after the smaller one: still the same result
    xb1 = torch.zeros_like(bt1)
    s_b1 = H1.solve_noalloc(bt1, xb1, **p1)
    _same_solve(s_b1, s_r1)
    assert np.array_equal(host(xb1), xr1)


def test_noalloc_refuses_what_it_cannot_hold(namg):
    A = poisson2d(400)  # 160 000 rows
    H = namg.Hierarchy(A, device=0)
    b = dev(np.random.default_rng(11).standard_normal(A.n))
    x = torch.zeros_like(b)
    # restart 128 in FP64: V and Z alone take 8 * 160 000 * (130 + 128) bytes = 330 MB > 256 MiB
    with pytest.raises(namg.NamgError) as e:
        H.solve_noalloc(b, x, restart=128)
    assert e.value.code == namg.E_INVALID and "static workspace" in str(e.value)
    with pytest.raises(namg.NamgError) as e:
        H.solve_noalloc(b, x, diagnostics=namg.DIAG_PHASE_TIMES)
    assert e.value.code == namg.E_INVALID
    with pytest.raises(namg.NamgError) as e:
        H.solve_noalloc(b, x, tri_mode=namg.TRI_DIRECT)
    assert e.value.code == namg.E_INVALID
    assert float(host(x).max()) == 0.0 and float(host(x).min()) == 0.0  # nothing was issued
    # the same system at restart 30 fits (80 MB) and matches namg_solve
    print(f"[noalloc] n {A.n} FP64 restart 30", flush=True)
    st = H.solve_noalloc(b, x, restart=30)
    xr = torch.zeros_like(b)
    sr = H.solve(b, xr, restart=30)
    _same_solve(st, sr)
    assert st["status"] == namg.OK
    assert np.array_equal(host(x), host(xr))
