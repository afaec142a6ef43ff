"""ctypes wrapper of the CPU FP64 oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the cpu_baseline leg of
bench.py. The library under paper_2112_14681_amd/ never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")

OK, NOT_CONVERGED, E_INVALID, E_ZERO_PIVOT, E_NONFINITE = 0, 1, -1, -2, -3
SMOOTH_PGS, SMOOTH_ILU0, SMOOTH_L1JAC = 0, 1, 2
TRI_NEUMANN, TRI_DIRECT = 0, 1
T_NEUMANN, T_DIRECT = 0, 1
PRECOND_NONE, PRECOND_AMG = 0, 1
STOP_RELRES, STOP_NRBE = 0, 1
ILU_KIND_ILU0, ILU_KIND_ILUT = 0, 1
COARSEN_RS, COARSEN_PMIS = 0, 1
PGS_FWD, PGS_BWD, GS_FWD, GS_BWD, ILU_NEUMANN, ILU_DIRECT, L1_JACOBI = range(7)


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (-O2 -ffp-contract=off, single-threaded)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
               _SRC, "-o", _LIB_PATH + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Params(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("max_iters", C.c_int), ("precond", C.c_int),
                ("smoother", C.c_int), ("tri_mode", C.c_int), ("inner_terms", C.c_int), ("gmres_T", C.c_int),
                ("pre_sweeps", C.c_int), ("post_sweeps", C.c_int), ("t_degree", C.c_int), ("stop_rule", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("cycles", C.c_int), ("precond_apps", C.c_int),
                ("relres_true", C.c_double), ("relres_est", C.c_double), ("nrbe", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.orc_setup.restype = C.c_void_p
        _lib.orc_loss_orth.restype = C.c_double
        _lib.orc_splitmix64.restype = C.c_ulonglong
        _lib.orc_uniform01.restype = C.c_double
        for name in ("orc_free", "orc_num_levels", "orc_level_info", "orc_level_export", "orc_vcycle",
                     "orc_solve"):
            getattr(_lib, name).argtypes = None
    return _lib


def _p(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleFailure(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def _check(code):
    if code < 0:
        raise OracleFailure(code)
    return code


def spmv(A, x):
    y = np.zeros(A.n)
    _check(lib().orc_spmv(A.n, _p(_i32(A.rowptr), C.c_int), _p(_i32(A.colind), C.c_int),
                          _p(_f64(A.vals), C.c_double), _p(_f64(x), C.c_double), _p(y, C.c_double)))
    return y


def strength(A, theta):
    srp = np.zeros(A.n + 1, np.int32)
    sci = np.zeros(max(A.nnz, 1), np.int32)
    _check(lib().orc_strength(A.n, _p(_i32(A.rowptr), C.c_int), _p(_i32(A.colind), C.c_int),
                              _p(_f64(A.vals), C.c_double), C.c_double(theta), _p(srp, C.c_int),
                              _p(sci, C.c_int)))
    return srp, sci[: srp[-1]].copy()


def coarsen(A, theta):
    cf = np.zeros(A.n, np.int8)
    _check(lib().orc_coarsen(A.n, _p(_i32(A.rowptr), C.c_int), _p(_i32(A.colind), C.c_int),
                             _p(_f64(A.vals), C.c_double), C.c_double(theta), _p(cf, C.c_int8)))
    return cf


def ilu0(A):
    out = np.zeros(A.nnz)
    _check(lib().orc_ilu0(A.n, _p(_i32(A.rowptr), C.c_int), _p(_i32(A.colind), C.c_int),
                          _p(_f64(A.vals), C.c_double), _p(out, C.c_double)))
    return out


def splitmix64(seed, k):
    return int(lib().orc_splitmix64(C.c_ulonglong(seed), C.c_ulonglong(k)))


def uniform01(seed, i):
    return float(lib().orc_uniform01(C.c_ulonglong(seed), C.c_longlong(i)))


def ilut(A, droptol, lfil):
    """ILUT(droptol, lfil) factors as a CSR holding L \\ U (strict lower = L_s, the rest = U)."""
    from workloads import CSR  # input container only

    n = A.n
    cap = n * min(n, 2 * lfil + 1)
    rp, ci, v = np.zeros(n + 1, np.int32), np.zeros(cap, np.int32), np.zeros(cap)
    nnz = C.c_longlong()
    _check(lib().orc_ilut(n, _p(_i32(A.rowptr), C.c_int), _p(_i32(A.colind), C.c_int), _p(_f64(A.vals), C.c_double),
                          C.c_double(droptol), lfil, C.c_longlong(cap), _p(rp, C.c_int), _p(ci, C.c_int), _p(v, C.c_double),
                          C.byref(nnz)))
    return CSR(n, rp, ci[: nnz.value].copy(), v[: nnz.value].copy())


def smooth_ilut(A, droptol, lfil, t, b, x, direct=False):
    xo = _f64(x).copy()
    _check(lib().orc_smooth_ilut(A.n, _p(_i32(A.rowptr), C.c_int), _p(_i32(A.colind), C.c_int),
                                 _p(_f64(A.vals), C.c_double), C.c_double(droptol), lfil, int(direct), t,
                                 _p(_f64(b), C.c_double), _p(xo, C.c_double)))
    return xo


def smooth(A, kind, t, b, x):
    xo = _f64(x).copy()
    _check(lib().orc_smooth(A.n, _p(_i32(A.rowptr), C.c_int), _p(_i32(A.colind), C.c_int),
                            _p(_f64(A.vals), C.c_double), kind, t, _p(_f64(b), C.c_double),
                            _p(xo, C.c_double)))
    return xo


@dataclass
class LevelExport:
    cf: np.ndarray | None
    A: object
    P: object | None


class Hierarchy:
    """Oracle AMG hierarchy (strength, RS first pass, classical P, Galerkin RAP, ILU(0), dense LU)."""

    def __init__(self, A, theta=0.25, max_levels=25, max_coarse=50, ilu_levels=1, ilu_kind=ILU_KIND_ILU0,
                 ilut_droptol=1e-2, ilut_lfil=5, agg_levels=0, coarsen=COARSEN_RS, seed=0):
        from workloads import CSR  # input container only

        self._CSR = CSR
        self.n = A.n
        self._rp, self._ci, self._v = _i32(A.rowptr), _i32(A.colind), _f64(A.vals)
        st = C.c_int(0)
        h = lib().orc_setup(A.n, _p(self._rp, C.c_int), _p(self._ci, C.c_int), _p(self._v, C.c_double),
                            C.c_double(theta), max_levels, max_coarse, ilu_levels, ilu_kind,
                            C.c_double(ilut_droptol), ilut_lfil, agg_levels, coarsen, C.c_ulonglong(seed),
                            C.byref(st))
        if st.value != 0 or not h:
            raise OracleFailure(st.value)
        self.h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.orc_free(h)
            self.h = None

    @property
    def levels(self) -> int:
        return lib().orc_num_levels(self.h)

    def level(self, l) -> LevelExport:
        n, na, npp, nc = C.c_int(), C.c_longlong(), C.c_longlong(), C.c_int()
        _check(lib().orc_level_info(self.h, l, C.byref(n), C.byref(na), C.byref(npp), C.byref(nc)))
        n = n.value
        last = l == self.levels - 1
        cf = None if last else np.zeros(n, np.int8)
        Arp, Aci, Av = np.zeros(n + 1, np.int32), np.zeros(na.value, np.int32), np.zeros(na.value)
        if last:
            Prp = Pci = Pv = None
        else:
            Prp, Pci, Pv = np.zeros(n + 1, np.int32), np.zeros(npp.value, np.int32), np.zeros(npp.value)
        _check(lib().orc_level_export(self.h, l, _p(cf, C.c_int8), _p(Arp, C.c_int), _p(Aci, C.c_int),
                                      _p(Av, C.c_double), _p(Prp, C.c_int), _p(Pci, C.c_int),
                                      _p(Pv, C.c_double)))
        A = self._CSR(n, Arp, Aci, Av)
        P = None
        if not last:
            import scipy.sparse as sp

            P = sp.csr_matrix((Pv, Pci, Prp), shape=(n, nc.value))
        return LevelExport(cf, A, P)

    def vcycle(self, b, smoother=SMOOTH_PGS, tri_mode=TRI_NEUMANN, t=2, nu1=1, nu2=1):
        x = np.zeros(self.n)
        _check(lib().orc_vcycle(self.h, smoother, tri_mode, t, nu1, nu2, _p(_f64(b), C.c_double),
                                _p(x, C.c_double)))
        return x

    def solve(self, b, x0=None, tol=1e-8, restart=30, max_iters=1000, precond=PRECOND_AMG,
              smoother=SMOOTH_PGS, tri_mode=TRI_NEUMANN, t=2, gmres_T=T_NEUMANN, nu1=1, nu2=1,
              capture=False, t_degree=1, stop_rule=STOP_RELRES):
        x = np.zeros(self.n) if x0 is None else _f64(x0).copy()
        p = Params(tol, restart, max_iters, precond, smoother, tri_mode, t, gmres_T, nu1, nu2, t_degree, stop_rule)
        st = Stats()
        cap = 4096
        hist = np.zeros(cap)
        cyc = np.zeros(cap)
        hl, cl, k = C.c_int(), C.c_int(), C.c_int(0)
        cV = cZ = cH = None
        if capture:
            cV = np.zeros((restart + 2, self.n))
            cZ = np.zeros((restart, self.n))
            cH = np.zeros((restart, restart + 1))
        code = lib().orc_solve(self.h, _p(_f64(b), C.c_double), _p(x, C.c_double), C.byref(p), C.byref(st),
                               _p(hist, C.c_double), cap, C.byref(hl), _p(cyc, C.c_double), cap,
                               C.byref(cl), _p(cV, C.c_double), _p(cZ, C.c_double), _p(cH, C.c_double),
                               C.byref(k) if capture else None)
        _check(code)
        out = {
            "x": x,
            "status": st.status,
            "iters": st.iters,
            "cycles": st.cycles,
            "precond_apps": st.precond_apps,
            "relres_true": st.relres_true,
            "relres_est": st.relres_est,
            "nrbe": st.nrbe,
            "hist": hist[: min(hl.value, cap)].copy(),
            "cycle_relres": cyc[: min(cl.value, cap)].copy(),
        }
        if capture:
            kk = k.value
            out["k"] = kk
            out["V"] = cV[: kk + 1].T.copy()
            out["Z"] = cZ[:kk].T.copy()
            out["H"] = cH[:kk, : kk + 1].T.copy()
        return out


def loss_orth(V):
    V = np.asfortranarray(V, dtype=np.float64)
    n, k = V.shape
    flat = np.ascontiguousarray(V.T)
    return lib().orc_loss_orth(n, k, _p(flat, C.c_double))
