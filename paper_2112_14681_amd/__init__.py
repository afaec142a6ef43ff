"""namg: Neumann-series GMRES + classical AMG on AMD Instinct MI355X (gfx950).

Thin ctypes binding of libnamg.so (include/namg.h). It only marshals arguments: every step of the solve
runs in the library's HIP kernels. Device vectors are torch tensors (float64, contiguous, on the
hierarchy's device); the stream is torch's current stream. There is no CPU fallback: if the compiled
library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnamg.so")

OK, NOT_CONVERGED, PENDING = 0, 1, 2
E_INVALID, E_ZERO_PIVOT, E_NONFINITE, E_NOMEM, E_HIP, E_BUDGET, E_NODEVICE = -1, -2, -3, -4, -5, -6, -7
FP64, FP32_PRECOND = 0, 1
SMOOTH_PGS, SMOOTH_ILU0, SMOOTH_L1JAC = 0, 1, 2
TRI_NEUMANN, TRI_DIRECT = 0, 1
T_NEUMANN, T_DIRECT = 0, 1
STOP_RELRES, STOP_NRBE = 0, 1
ILU0, ILUT = 0, 1
COARSEN_RS, COARSEN_PMIS = 0, 1
DIAG_LOSS_ORTH, DIAG_PHASE_TIMES = 1, 2
OP_SPMV, OP_RESIDUAL, OP_SMOOTH_PRE, OP_SMOOTH_POST, OP_RESTRICT, OP_PROLONG, OP_COARSE, OP_SPMV64 = range(8)
MAX_LEVELS = 32
NOALLOC_SCRATCH_BYTES = 256 << 20  # NAMG_NOALLOC_SCRATCH_BYTES

KF_NONE, KF_NEUMANN, KF_RESIDUAL, KF_SPMV, KF_PROLONG, KF_GMRES_SPMV, KF_MULTIDOT, KF_PROJECT, KF_TRI = range(9)

EXPORTED = (
    "namg_default_setup_params", "namg_default_solve_params", "namg_setup", "namg_solve", "namg_solve_noalloc",
    "namg_vcycle",
    "namg_apply", "namg_profile_kernel", "namg_profile_read", "namg_hier_info", "namg_level_sizes",
    "namg_export_level", "namg_export_ilu", "namg_ilu_diagnostics", "namg_tri_jacobi_residuals",
    "namg_us_powers", "namg_destroy", "namg_last_error", "namg_default_server_params", "namg_server_create",
    "namg_server_submit", "namg_server_poll", "namg_server_wait", "namg_server_stats", "namg_server_clock",
    "namg_server_destroy",
)


class SetupParams(C.Structure):
    _fields_ = [("theta", C.c_double), ("max_levels", C.c_int), ("max_coarse", C.c_int), ("precision", C.c_int),
                ("ilu_levels", C.c_int), ("device", C.c_int), ("ilu_kind", C.c_int), ("ilut_lfil", C.c_int),
                ("ilut_droptol", C.c_double), ("agg_levels", C.c_int), ("coarsen", C.c_int), ("seed", C.c_uint64)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("max_iters", C.c_int), ("smoother", C.c_int),
                ("tri_mode", C.c_int), ("inner_terms", C.c_int), ("gmres_T", C.c_int), ("pre_sweeps", C.c_int),
                ("post_sweeps", C.c_int), ("t_degree", C.c_int), ("stop_rule", C.c_int), ("diagnostics", C.c_int),
                ("res_hist", C.POINTER(C.c_double)), ("res_hist_cap", C.c_int)]


class IluDiag(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_lower", C.c_int64), ("nnz_upper", C.c_int64), ("max_row_upper", C.c_int),
                ("ruiz_iters", C.c_int), ("dep_L", C.c_double), ("dep_U", C.c_double), ("nu", C.c_double),
                ("norm2_Us", C.c_double), ("th1_bound", C.c_double), ("th3_bound", C.c_double),
                ("delta", C.c_double), ("th4_bound", C.c_double), ("dep_U_ruiz", C.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("cycles", C.c_int), ("precond_apps", C.c_int),
                ("relres_true", C.c_double), ("relres_est", C.c_double), ("nrbe", C.c_double),
                ("ms_total", C.c_double), ("alg_bytes", C.c_double), ("loss_orth", C.c_double),
                ("ms_vcycle", C.c_double), ("ms_spmv", C.c_double), ("ms_ortho", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("alg_bytes", C.c_double)]


class HierInfo(C.Structure):
    _fields_ = [("levels", C.c_int), ("n", C.c_int32 * MAX_LEVELS), ("nnz", C.c_int64 * MAX_LEVELS),
                ("op_complexity", C.c_double), ("grid_complexity", C.c_double), ("device_bytes", C.c_int64)]


class ServerParams(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_inflight", C.c_int), ("setup_threads", C.c_int), ("device", C.c_int),
                ("precision", C.c_int), ("solve", SolveParams)]


class RequestTimes(C.Structure):
    _fields_ = [("submit", C.c_double), ("setup_start", C.c_double), ("setup_done", C.c_double),
                ("admitted", C.c_double), ("done", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerCounters(C.Structure):
    _fields_ = [(name, C.c_int64) for name in ("submitted", "completed", "failed", "inflight", "waiting", "ticks",
                                               "launches", "device_bytes_in_use", "peak_device_bytes",
                                               "peak_inflight", "footprint_mismatches",
                                               "peak_setup_device_bytes")]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class NamgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"namg error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                          " (the HIP library is required; there is no CPU fallback)")
    # One HIP runtime per process: torch ships its own, and a second one loaded first (the system's, which
    # the library links) finds no device once torch has initialised its copy. Importing torch first makes
    # the library resolve to torch's already-loaded runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, i32p, f64p, i8p, i64p = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int8), \
        C.POINTER(C.c_int64)
    lib.namg_setup.argtypes = [C.c_int32, i32p, i32p, f64p, C.POINTER(SetupParams), C.POINTER(vp)]
    lib.namg_solve.argtypes = [vp, vp, vp, C.POINTER(SolveParams), vp, C.POINTER(SolveStats)]
    lib.namg_solve_noalloc.argtypes = [vp, vp, vp, C.POINTER(SolveParams), vp, C.POINTER(SolveStats)]
    lib.namg_vcycle.argtypes = [vp, vp, vp, C.POINTER(SolveParams), vp]
    lib.namg_apply.argtypes = [vp, C.c_int, C.c_int, C.POINTER(SolveParams), vp, vp, vp, vp]
    lib.namg_profile_kernel.argtypes = [vp, C.c_int, C.c_int, C.c_int]
    lib.namg_profile_read.argtypes = [vp, C.POINTER(KernelProfile)]
    lib.namg_hier_info.argtypes = [vp, C.POINTER(HierInfo)]
    lib.namg_level_sizes.argtypes = [vp, C.c_int, i32p, i64p, i64p, i32p]
    lib.namg_export_level.argtypes = [vp, C.c_int, i8p, i32p, i32p, f64p, i32p, i32p, f64p]
    lib.namg_destroy.argtypes = [vp]
    lib.namg_destroy.restype = None
    lib.namg_last_error.restype = C.c_char_p
    lib.namg_default_setup_params.argtypes = [C.POINTER(SetupParams)]
    lib.namg_default_solve_params.argtypes = [C.POINTER(SolveParams)]
    lib.namg_default_server_params.argtypes = [C.POINTER(ServerParams)]
    lib.namg_server_create.argtypes = [C.POINTER(ServerParams), C.POINTER(vp)]
    lib.namg_server_submit.argtypes = [vp, C.c_int32, i32p, i32p, f64p, f64p, C.POINTER(SetupParams),
                                       C.POINTER(SolveParams), C.POINTER(C.c_uint64)]
    lib.namg_server_poll.argtypes = [vp, C.c_uint64, f64p, C.POINTER(SolveStats), C.POINTER(RequestTimes)]
    lib.namg_server_wait.argtypes = [vp, C.c_uint64, f64p, C.POINTER(SolveStats), C.POINTER(RequestTimes)]
    lib.namg_server_stats.argtypes = [vp, C.POINTER(ServerCounters)]
    lib.namg_server_clock.argtypes = [vp]
    lib.namg_server_clock.restype = C.c_double
    lib.namg_server_destroy.argtypes = [vp]
    lib.namg_server_destroy.restype = None
    return lib


_lib = _load()


def lib():
    return _lib


def _check(code):
    if code < 0:
        raise NamgError(code, _lib.namg_last_error().decode())
    return code


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def setup_params(**kw) -> SetupParams:
    p = SetupParams()
    _lib.namg_default_setup_params(C.byref(p))
    _set_fields(p, kw)
    return p


def solve_params(**kw) -> SolveParams:
    p = SolveParams()
    _lib.namg_default_solve_params(C.byref(p))
    _set_fields(p, kw)
    return p


def _set_fields(p, kw):
    """Set named fields of a parameter struct; an unknown name is an error, not a silent attribute."""
    names = {f[0] for f in type(p)._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"{type(p).__name__} has no field {k!r}")
        setattr(p, k, v)


def _dev_ptr(t, n=None):
    """Device pointer of a contiguous float64 torch tensor (checked)."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 device tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} entries, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Hierarchy:
    """An AMG hierarchy set up from a host CSR matrix (namg_setup); owns its device memory."""

    def __init__(self, A, **params):
        rp = np.ascontiguousarray(A.rowptr, dtype=np.int32)
        ci = np.ascontiguousarray(A.colind, dtype=np.int32)
        v = np.ascontiguousarray(A.vals, dtype=np.float64)
        self.n = int(A.n)
        self.params = setup_params(**params)
        h = C.c_void_p()
        _check(_lib.namg_setup(self.n, _ptr(rp, C.c_int32), _ptr(ci, C.c_int32), _ptr(v, C.c_double),
                               C.byref(self.params), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.namg_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = HierInfo()
        _check(_lib.namg_hier_info(self.h, C.byref(inf)))
        L = inf.levels
        return {"levels": L, "n": list(inf.n[:L]), "nnz": list(inf.nnz[:L]), "op_complexity": inf.op_complexity,
                "grid_complexity": inf.grid_complexity, "device_bytes": inf.device_bytes}

    def level_sizes(self, level):
        n, na, npp, nc = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(_lib.namg_level_sizes(self.h, level, C.byref(n), C.byref(na), C.byref(npp), C.byref(nc)))
        return n.value, na.value, npp.value, nc.value

    def export_level(self, level):
        """Host copies (cf, A as CSR triple, P as CSR triple or None)."""
        n, na, npp, nc = self.level_sizes(level)
        last = npp == 0 and nc == 0
        cf = None if last else np.zeros(n, np.int8)
        Arp, Aci, Av = np.zeros(n + 1, np.int32), np.zeros(na, np.int32), np.zeros(na)
        Prp = Pci = Pv = None
        if not last:
            Prp, Pci, Pv = np.zeros(n + 1, np.int32), np.zeros(npp, np.int32), np.zeros(npp)
        _check(_lib.namg_export_level(self.h, level, _ptr(cf, C.c_int8), _ptr(Arp, C.c_int32), _ptr(Aci, C.c_int32),
                                      _ptr(Av, C.c_double), _ptr(Prp, C.c_int32), _ptr(Pci, C.c_int32),
                                      _ptr(Pv, C.c_double)))
        return {"cf": cf, "A": (Arp, Aci, Av), "P": None if last else (Prp, Pci, Pv, nc)}

    def export_ilu(self, level):
        """Host copies of the ILU smoother factors: L_s and U_s = D_U^{-1} strict(U) as CSR triples, 1/u_ii."""
        nl, nu = C.c_int64(), C.c_int64()
        _check(_lib.namg_export_ilu(self.h, level, C.byref(nl), C.byref(nu), None, None, None, None, None, None, None))
        n = self.level_sizes(level)[0]
        L = (np.zeros(n + 1, np.int32), np.zeros(nl.value, np.int32), np.zeros(nl.value))
        U = (np.zeros(n + 1, np.int32), np.zeros(nu.value, np.int32), np.zeros(nu.value))
        dinv = np.zeros(n)
        _check(_lib.namg_export_ilu(self.h, level, C.byref(nl), C.byref(nu), _ptr(L[0], C.c_int32),
                                    _ptr(L[1], C.c_int32), _ptr(L[2], C.c_double), _ptr(U[0], C.c_int32),
                                    _ptr(U[1], C.c_int32), _ptr(U[2], C.c_double), _ptr(dinv, C.c_double)))
        return {"L": L, "U": U, "dinv": dinv}

    def ilu_diagnostics(self, level, power_iters=100, ruiz_max_iters=20, ruiz_tol=1e-8) -> dict:
        """Non-normality of the level's ILU factors (namg_ilu_diagnostics)."""
        d = IluDiag()
        _check(_lib.namg_ilu_diagnostics(self.h, level, power_iters, ruiz_max_iters, C.c_double(ruiz_tol),
                                         C.byref(d)))
        return d.as_dict()

    def tri_jacobi_residuals(self, level, b, iters) -> tuple:
        """(||b - L y|| / ||b||, ||y - U v|| / ||y||) after `iters` Jacobi iterations (host b)."""
        bb = np.ascontiguousarray(b, dtype=np.float64)
        if bb.shape != (self.level_sizes(level)[0],):
            raise ValueError("b must have n_l entries")
        rl, ru = C.c_double(), C.c_double()
        _check(_lib.namg_tri_jacobi_residuals(self.h, level, _ptr(bb, C.c_double), iters, C.byref(rl), C.byref(ru)))
        return rl.value, ru.value

    def us_powers(self, level, pmax, power_iters=200) -> dict:
        """max |(U_s^p)_ij|, ||U_s^p||_2 (power-iteration estimate) and nnz(U_s^p) for p = 1..pmax."""
        ma, n2 = np.zeros(pmax), np.zeros(pmax)
        nz = np.zeros(pmax, dtype=np.int64)
        _check(_lib.namg_us_powers(self.h, level, pmax, power_iters, _ptr(ma, C.c_double), _ptr(n2, C.c_double),
                                   _ptr(nz, C.c_int64)))
        return {"max_abs": ma, "norm2": n2, "nnz": nz}

    def solve(self, b, x, stream=None, history=False, **params) -> dict:
        """namg_solve on device tensors b (read) and x (initial guess in, solution out). history=True also
        returns the residual estimate after every iteration ("hist")."""
        return self._solve(_lib.namg_solve, b, x, stream, history, params)

    def solve_noalloc(self, b, x, stream=None, history=False, **params) -> dict:
        """namg_solve_noalloc: the same solve with the Krylov workspace in the library's static per-device
        array (NOALLOC_SCRATCH_BYTES); no device allocation."""
        return self._solve(_lib.namg_solve_noalloc, b, x, stream, history, params)

    def _solve(self, entry, b, x, stream, history, params) -> dict:
        p = solve_params(**params)
        hist = None
        if history:
            hist = np.zeros(max(p.max_iters, 1))
            p.res_hist = _ptr(hist, C.c_double)
            p.res_hist_cap = hist.size
        st = SolveStats()
        code = _check(entry(self.h, _dev_ptr(b, self.n), _dev_ptr(x, self.n), C.byref(p), _stream(stream),
                            C.byref(st)))
        out = st.as_dict()
        out["status"] = code
        if history:
            out["hist"] = hist[: st.iters].copy()
        return out

    def vcycle(self, b, x, stream=None, **params):
        p = solve_params(**params)
        _check(_lib.namg_vcycle(self.h, _dev_ptr(b, self.n), _dev_ptr(x, self.n), C.byref(p), _stream(stream)))

    def profile_kernel(self, family, level=-1, every=1):
        """Time later launches of a kernel family (hipEvents attached to the first and then every
        `every`-th matching dispatch)."""
        _check(_lib.namg_profile_kernel(self.h, family, level, every))

    def profile_read(self) -> dict:
        kp = KernelProfile()
        _check(_lib.namg_profile_read(self.h, C.byref(kp)))
        return {"launches": kp.launches, "total_ms": kp.total_ms, "alg_bytes": kp.alg_bytes}

    def apply(self, level, op, in1, in2, out, stream=None, **params):
        p = solve_params(**params)
        _check(_lib.namg_apply(self.h, level, op, C.byref(p), _dev_ptr(in1), _dev_ptr(in2), _dev_ptr(out),
                               _stream(stream)))


def server_params(solve=None, **kw) -> ServerParams:
    p = ServerParams()
    _lib.namg_default_server_params(C.byref(p))
    _set_fields(p, kw)
    _set_fields(p.solve, solve or {})
    return p


class Server:
    """Continuous-batching request server (namg_server_*): submit host systems, poll or wait for x."""

    def __init__(self, solve=None, **params):
        self.params = server_params(solve, **params)
        h = C.c_void_p()
        _check(_lib.namg_server_create(C.byref(self.params), C.byref(h)))
        self.h = h
        self._sizes = {}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.namg_server_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self) -> float:
        return _lib.namg_server_clock(self.h)

    def submit(self, A, b, solve=None, **setup) -> int:
        """Queue A x = b with setup parameters `setup`; `solve` (a dict of solve parameters) replaces the
        server's default solve parameters for this request."""
        rp = np.ascontiguousarray(A.rowptr, dtype=np.int32)
        ci = np.ascontiguousarray(A.colind, dtype=np.int32)
        v = np.ascontiguousarray(A.vals, dtype=np.float64)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        sp = setup_params(**setup)
        sv = None
        if solve is not None:
            sv = SolveParams.from_buffer_copy(self.params.solve)
            _set_fields(sv, solve)
        t = C.c_uint64()
        _check(_lib.namg_server_submit(self.h, int(A.n), _ptr(rp, C.c_int32), _ptr(ci, C.c_int32), _ptr(v, C.c_double),
                                       _ptr(bb, C.c_double), C.byref(sp), C.byref(sv) if sv is not None else None,
                                       C.byref(t)))
        self._sizes[t.value] = int(A.n)
        return t.value

    def _result(self, fn, ticket):
        n = self._sizes[ticket]
        x = np.zeros(n)
        st, tm = SolveStats(), RequestTimes()
        code = fn(self.h, ticket, _ptr(x, C.c_double), C.byref(st), C.byref(tm))
        if code == PENDING:
            return None
        del self._sizes[ticket]
        if code < 0:
            raise NamgError(code, _lib.namg_last_error().decode())
        out = st.as_dict()
        out.update(status=code, x=x, times=tm.as_dict())
        return out

    def poll(self, ticket):
        """None while pending, else the result dict (x, statistics, times)."""
        return self._result(_lib.namg_server_poll, ticket)

    def wait(self, ticket):
        return self._result(_lib.namg_server_wait, ticket)

    def stats(self) -> dict:
        c = ServerCounters()
        _check(_lib.namg_server_stats(self.h, C.byref(c)))
        return c.as_dict()
