"""GPU parity of the device setup (PMIS coarsening, BAMG direct interpolation, Galerkin products; Section
5.1) against the oracle's PMIS hierarchy: every level's C/F splitting, P and coarse operator bit for bit,
then solves on that hierarchy with the oracle's iterations and iterate."""
import time

import numpy as np
import pytest

import oracle as O
from workloads import config_system, poisson3d, random_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def namg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_14681_amd as m

    return m


def _compare(namg, A, seed, **kw):
    H = namg.Hierarchy(A, device=0, coarsen=namg.COARSEN_PMIS, seed=seed, **kw)
    G = O.Hierarchy(A, coarsen=O.COARSEN_PMIS, seed=seed, **kw)
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
    return H, G, info


@pytest.mark.parametrize("name,N,seed", [("c1", None, 0), ("c2", 20, 7), ("c3", 18, 1), ("c4r", 14, 3),
                                         ("c4n", 17, 2**40 + 5)])
def test_device_pmis_setup_bit_exact(namg, name, N, seed):
    A, _, _ = config_system(name, N)
    _compare(namg, A, seed)


def test_device_pmis_setup_edge_cases(namg):
    """A nonsymmetric random matrix, a 64^3 grid (262 144 rows: many blocks, several hundred PMIS
    rounds in total), a system small enough for one level, and a 1 x 1 system."""
    _compare(namg, random_csr(400, 7, 5), 9, max_coarse=10)
    _, _, info = _compare(namg, poisson3d(64), 0)
    assert info["levels"] >= 5
    H, _, info = _compare(namg, poisson3d(3), 0)
    assert info["levels"] == 1
    from workloads import CSR

    one = CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    _compare(namg, one, 0)


def _product_row_classes(G):
    """Over the oracle hierarchy's products A P and R (A P): rows whose X row has more than 64 entries, rows
    with at most 64 products, and the others (the device setup's three kernels' shares)."""
    cls = {"le64": 0, "gt64": 0, "long_x": 0}

    def count(Xrp, Xci, ylen):
        for i in range(len(Xrp) - 1):
            cols = Xci[Xrp[i]:Xrp[i + 1]]
            key = "long_x" if len(cols) > 64 else ("le64" if ylen[cols].sum() <= 64 else "gt64")
            cls[key] += 1

    for l in range(G.levels - 1):
        g = G.level(l)
        P = g.P.tocsr()
        count(g.A.rowptr, g.A.colind, np.diff(P.indptr))
        R = P.T.tocsr()
        AP = (g.A.to_scipy() @ P).tocsr()
        count(R.indptr, R.indices, np.diff(AP.indptr))
    return cls


@pytest.mark.parametrize("n,per_row,seed", [(600, 24, 11), (800, 12, 4)])
def test_device_sparse_products_all_row_classes(namg, n, per_row, seed):
    """Random nonsymmetric matrices whose Galerkin products have rows of every kind the device setup
    distinguishes (at most 64 products: one wavefront per row; more: a per-row table; more than 64 entries
    in the left factor's row: the table too): every level still equals the oracle's bit for bit."""
    A = random_csr(n, per_row, seed)
    _, G, _ = _compare(namg, A, 9, max_coarse=10)
    cls = _product_row_classes(G)
    assert min(cls.values()) > 0, cls


@pytest.mark.parametrize("name,N,kw", [("c2", 24, dict(smoother=1, inner_terms=3)),
                                       ("c3", 20, dict(smoother=0, inner_terms=2))])
def test_solve_on_device_pmis_hierarchy(namg, name, N, kw):
    """GMRES + AMG on the device-built PMIS hierarchy: the oracle's iterations on its PMIS hierarchy,
    x within 1e-10, true relative residual 1e-8; the FP32 preconditioner within two iterations."""
    A, b, _ = config_system(name, N)
    H, G, _ = _compare(namg, A, 5)
    ref = G.solve(b, smoother=kw["smoother"], t=kw["inner_terms"])
    bt = torch.from_numpy(b).to("cuda:0")
    xt = torch.zeros_like(bt)
    st = H.solve(bt, xt, **kw)
    x = xt.cpu().numpy()
    assert st["status"] == namg.OK and st["iters"] == ref["iters"]
    gap = np.abs(x - ref["x"]).max() / np.abs(ref["x"]).max()
    assert gap <= 1e-10, gap
    assert np.linalg.norm(b - O.spmv(A, x)) <= 1e-8 * np.linalg.norm(b)
    H32 = namg.Hierarchy(A, device=0, coarsen=namg.COARSEN_PMIS, seed=5, precision=namg.FP32_PRECOND)
    xt.zero_()
    st = H32.solve(bt, xt, **kw)
    assert st["status"] == namg.OK and abs(st["iters"] - ref["iters"]) <= 2


def test_device_setup_time_and_server(namg):
    """Device setup of a 94^3 variable-coefficient system against the host RS setup (printed), and a
    served request with PMIS setup parameters equal to namg_solve on the same hierarchy."""
    from workloads import varcoef3d

    A, b = varcoef3d(94, 0.5, 11)
    t0 = time.perf_counter()
    Hd = namg.Hierarchy(A, device=0, coarsen=namg.COARSEN_PMIS, ilu_levels=0)
    t1 = time.perf_counter()
    Hh = namg.Hierarchy(A, device=-1, ilu_levels=0)
    t2 = time.perf_counter()
    print(f"setup of {A.n} rows: device PMIS {1e3 * (t1 - t0):.0f} ms "
          f"(op. complexity {Hd.info()['op_complexity']:.2f}), host RS {1e3 * (t2 - t1):.0f} ms "
          f"(op. complexity {Hh.info()['op_complexity']:.2f})")
    Hd.close()
    A, b, _ = config_system("c3", 16)
    solve = dict(smoother=0, inner_terms=2)
    srv = namg.Server(solve=solve, max_inflight=2, setup_threads=2, precision=0)
    tickets = [srv.submit(A, b, coarsen=namg.COARSEN_PMIS, seed=4) for _ in range(3)]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    H = namg.Hierarchy(A, device=0, coarsen=namg.COARSEN_PMIS, seed=4)
    bt = torch.from_numpy(b).to("cuda:0")
    xt = torch.zeros_like(bt)
    st = H.solve(bt, xt, **solve)
    for r in res:
        assert r["status"] == namg.OK and r["iters"] == st["iters"]
        assert np.array_equal(r["x"], xt.cpu().numpy())


@pytest.mark.parametrize("precision", [0, 1])
def test_device_packing_matches_host_packing(namg, precision, monkeypatch):
    """Levels built on the device are packed into the solve-phase layouts on the device; with
    NAMG_HOST_PACK set the same hierarchy is packed on the host. Both give the same V-cycle and the same
    solve bit for bit (FP64 and FP32 layouts, SELL-64 and lane-group levels, 16-bit and 32-bit columns:
    the random relabelling keeps 32-bit columns on the finest level)."""
    for name, N, kw, ilu in (("c2", 24, dict(smoother=1, inner_terms=3), 1),
                             ("c3", 20, dict(smoother=0, inner_terms=2), 0),
                             ("c4r", 18, dict(smoother=0, inner_terms=2), 0)):
        A, b, _ = config_system(name, N)
        setup = dict(device=0, coarsen=namg.COARSEN_PMIS, seed=3, precision=precision, ilu_levels=ilu)
        bt = torch.from_numpy(b).to("cuda:0")
        out = []
        for host_pack in (False, True):
            if host_pack:
                monkeypatch.setenv("NAMG_HOST_PACK", "1")
            else:
                monkeypatch.delenv("NAMG_HOST_PACK", raising=False)
            H = namg.Hierarchy(A, **setup)
            zt = torch.empty_like(bt)
            H.vcycle(bt, zt, **kw)
            xt = torch.zeros_like(bt)
            st = H.solve(bt, xt, **kw)
            torch.cuda.synchronize()
            out.append((zt.cpu().numpy(), xt.cpu().numpy(), st["iters"], H.info()["device_bytes"]))
            H.close()
        monkeypatch.delenv("NAMG_HOST_PACK", raising=False)
        (z0, x0, i0, b0), (z1, x1, i1, b1) = out
        assert np.array_equal(z0, z1), name
        assert np.array_equal(x0, x1) and i0 == i1, name
        assert b0 == b1, name


@pytest.mark.parametrize("smoother", [0, 1])
def test_direct_comparator_on_device_built_hierarchy(namg, smoother, monkeypatch):
    """A hierarchy packed on the device keeps no host copy of the scaled triangles; the direct-triangular
    comparator derives them on its first use. Its V-cycle and solve equal those of the same hierarchy
    packed on the host (where the setup builds the copies), bit for bit, for polynomial GS and ILU(0)."""
    A, b, _ = config_system("c2", 16)
    setup = dict(device=0, coarsen=namg.COARSEN_PMIS, seed=5, ilu_levels=1)
    kw = dict(smoother=smoother, tri_mode=namg.TRI_DIRECT, inner_terms=2)
    bt = torch.from_numpy(b).to("cuda:0")
    out = []
    for host_pack in (False, True):
        if host_pack:
            monkeypatch.setenv("NAMG_HOST_PACK", "1")
        else:
            monkeypatch.delenv("NAMG_HOST_PACK", raising=False)
        H = namg.Hierarchy(A, **setup)
        monkeypatch.delenv("NAMG_HOST_PACK", raising=False)  # the hierarchy keeps the choice made at setup
        zt = torch.empty_like(bt)
        H.vcycle(bt, zt, **kw)
        xt = torch.zeros_like(bt)
        st = H.solve(bt, xt, **kw)
        torch.cuda.synchronize()
        out.append((zt.cpu().numpy(), xt.cpu().numpy(), st["iters"], st["status"]))
        H.close()
    (z0, x0, i0, s0), (z1, x1, i1, s1) = out
    assert s0 == namg.OK and s1 == namg.OK
    assert np.array_equal(z0, z1)
    assert np.array_equal(x0, x1) and i0 == i1
