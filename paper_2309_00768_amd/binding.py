"""ctypes binding of libst (argument marshalling only; every step runs in the library).

The library is ``paper_2309_00768_amd/libst.so`` (built by ``build.py``).  PyTorch
supplies device memory (the workspace and all vectors) and streams.  Importing
this module raises ``RuntimeError`` if the library is missing: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libst.so")

ST_OK, ST_ENOTCONV = 0, 1
ST_FP64, ST_FP32 = 0, 1
ST_INNER_AMG, ST_INNER_EXACT = 0, 1

BLOCK_IDS = {"Fu": 0, "Mu": 1, "B": 2, "Zj": 3, "ZA": 4, "Mj": 5, "KjA": 6, "Y": 7, "FA": 8,
             "MA": 9, "KA": 10, "Kp": 11, "Fp": 12, "C0": 13, "C1": 14, "C2": 15}


class StProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("nt", ctypes.c_int),
        ("dt", ctypes.c_double), ("mu", ctypes.c_double), ("eta", ctypes.c_double), ("mu0", ctypes.c_double),
        ("ubar", ctypes.POINTER(ctypes.c_double)), ("abar", ctypes.POINTER(ctypes.c_double)),
        ("jbar", ctypes.POINTER(ctypes.c_double)),
        ("precond_precision", ctypes.c_int), ("inner_mode", ctypes.c_int), ("inner_iters", ctypes.c_int),
        ("mass_iters", ctypes.c_int), ("cheb_degree", ctypes.c_int), ("fu_solver", ctypes.c_int),
        ("ca_solver", ctypes.c_int), ("max_restart", ctypes.c_int), ("sell_sigma", ctypes.c_int),
        ("adjoint", ctypes.c_int), ("j_lanes", ctypes.c_int), ("sweep_format", ctypes.c_int),
        ("single_stream", ctypes.c_int), ("sweep_chunk", ctypes.c_int), ("sweep_chain", ctypes.c_int),
        ("j_slabs", ctypes.c_int), ("sweep_fuse", ctypes.c_int),
        ("autotune", ctypes.c_int), ("sweep_lanes", ctypes.c_int),
        ("inner_reduction", ctypes.c_double), ("ca_reduction", ctypes.c_double),
        ("precond_variant", ctypes.c_int), ("time_parallel", ctypes.c_int), ("time_coarse_degree", ctypes.c_int),
    ]


ORTH = {"auto": 0, "cgs2": 1, "delayed": 2}


class StOpts(ctypes.Structure):
    _fields_ = [
        ("restart", ctypes.c_int), ("maxit", ctypes.c_int), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
        ("x0_given", ctypes.c_int), ("history_len", ctypes.c_int), ("history", ctypes.POINTER(ctypes.c_double)),
        ("orth", ctypes.c_int),
    ]


class StNlProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("nt", ctypes.c_int),
        ("dt", ctypes.c_double), ("mu", ctypes.c_double), ("eta", ctypes.c_double), ("mu0", ctypes.c_double),
        ("u_base", ctypes.POINTER(ctypes.c_double)), ("p_base", ctypes.POINTER(ctypes.c_double)),
        ("j_base", ctypes.POINTER(ctypes.c_double)), ("a_base", ctypes.POINTER(ctypes.c_double)),
        ("u_init", ctypes.POINTER(ctypes.c_double)), ("a_init", ctypes.POINTER(ctypes.c_double)),
        ("f", ctypes.POINTER(ctypes.c_double)), ("e", ctypes.POINTER(ctypes.c_double)),
    ]


ST_NEWTON_MAX = 32


class StInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
        ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double), ("precond_seconds", ctypes.c_double),
        ("jacobian_seconds", ctypes.c_double), ("jacobian_calls", ctypes.c_int), ("precond_calls", ctypes.c_int),
    ]


class StNewtonOpts(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int), ("atol", ctypes.c_double), ("linear", StOpts)]


class StNewtonInfo(ctypes.Structure):
    _fields_ = [
        ("newton_iterations", ctypes.c_int), ("converged", ctypes.c_int), ("linear_iterations_total", ctypes.c_int),
        ("linear_iterations", ctypes.c_int * ST_NEWTON_MAX), ("residual_norm", ctypes.c_double * (ST_NEWTON_MAX + 1)),
        ("seconds", ctypes.c_double), ("setup_seconds", ctypes.c_double),
    ]


EXPORTED = [
    "st_plan_create", "st_plan_workspace_size", "st_plan_sizes", "st_plan_export_block", "st_plan_export_jbar",
    "st_plan_solver_info", "st_plan_cheb_intervals", "st_plan_jacobian_slots",
    "st_plan_destroy", "st_create", "st_destroy", "st_apply_jacobian", "st_apply_jacobian_t",
    "st_apply_precond", "st_apply_precond_t", "st_apply_precond_noalloc", "st_apply_initial_coupling",
    "st_fgmres_solve", "st_adjoint_solve", "st_timestep_solve",
    "st_sizes", "st_tuning", "st_profile_kernel", "st_profile_read", "st_batch_create", "st_batch_workspace_size",
    "st_batch_upload", "st_batch_launch_counts",
    "st_fgmres_solve_batched", "st_batch_destroy",
    "st_nl_workspace_size", "st_nl_create", "st_nl_residual", "st_newton_solve", "st_nl_destroy",
    "st_error_string",
]


def _load(path=LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"libst not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "st_plan_create": ([ctypes.POINTER(StProblem), ctypes.POINTER(vp)], ctypes.c_int),
        "st_plan_workspace_size": ([vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "st_plan_sizes": ([vp, ip, ip], ctypes.c_int),
        "st_plan_export_block": ([vp, ctypes.c_int, ctypes.c_int, ip, ip, i64p, ip, ip, dp], ctypes.c_int),
        "st_plan_export_jbar": ([vp, dp], ctypes.c_int),
        "st_plan_solver_info": ([vp, ip, ip, dp, dp], ctypes.c_int),
        "st_plan_cheb_intervals": ([vp, ctypes.c_int, dp], ctypes.c_int),
        "st_plan_jacobian_slots": ([vp, i64p, ip], ctypes.c_int),
        "st_plan_destroy": ([vp], ctypes.c_int),
        "st_create": ([vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "st_destroy": ([vp], ctypes.c_int),
        "st_apply_jacobian": ([vp, vp, vp, vp], ctypes.c_int),
        "st_apply_jacobian_t": ([vp, vp, vp, vp], ctypes.c_int),
        "st_apply_precond": ([vp, vp, vp, vp], ctypes.c_int),
        "st_apply_precond_t": ([vp, vp, vp, vp], ctypes.c_int),
        "st_apply_precond_noalloc": ([vp, vp, vp, vp], ctypes.c_int),
        "st_apply_initial_coupling": ([vp, vp, vp, vp], ctypes.c_int),
        "st_fgmres_solve": ([vp, vp, vp, ctypes.POINTER(StOpts), ctypes.POINTER(StInfo), vp], ctypes.c_int),
        "st_adjoint_solve": ([vp, vp, vp, ctypes.POINTER(StOpts), ctypes.POINTER(StInfo), vp], ctypes.c_int),
        "st_timestep_solve": ([ctypes.POINTER(vp), ctypes.c_int, vp, vp, ctypes.POINTER(StOpts),
                               ctypes.POINTER(StInfo), vp], ctypes.c_int),
        "st_sizes": ([vp, i64p, ip, ip], ctypes.c_int),
        "st_tuning": ([vp, ip, ip, ip, ip, ip], ctypes.c_int),
        "st_profile_kernel": ([vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "st_profile_read": ([vp, dp, i64p, i64p], ctypes.c_int),
        "st_batch_create": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "st_batch_workspace_size": ([vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "st_batch_upload": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "st_batch_launch_counts": ([vp, i64p, i64p], ctypes.c_int),
        "st_fgmres_solve_batched": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(StOpts),
                                     ctypes.POINTER(StInfo), ip, vp], ctypes.c_int),
        "st_batch_destroy": ([vp], ctypes.c_int),
        "st_nl_workspace_size": ([ctypes.POINTER(StNlProblem), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "st_nl_create": ([ctypes.POINTER(StNlProblem), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "st_nl_residual": ([vp, vp, vp, vp], ctypes.c_int),
        "st_newton_solve": ([vp, ctypes.POINTER(StProblem), vp, ctypes.c_size_t, vp, ctypes.POINTER(StNewtonOpts),
                             ctypes.POINTER(StNewtonInfo), vp], ctypes.c_int),
        "st_nl_destroy": ([vp], ctypes.c_int),
        "st_error_string": ([ctypes.c_int], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


class StError(RuntimeError):
    def __init__(self, code, what):
        msg = lib().st_error_string(code).decode()
        super().__init__(f"{what}: {msg} (status {code})")
        self.code = code


def _check(code, what):
    if code < 0:
        raise StError(code, what)
    return code


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Plan:
    """Host-side setup of one space-time system (``st_plan_create``)."""

    def __init__(self, n, nt, dt, mu, eta, mu0, ubar, abar, jbar=None, precision="fp64", inner="amg",
                 inner_iters=0, mass_iters=0, cheb_degree=0, max_restart=0, sell_sigma=0, adjoint=False,
                 fu_solver=0, ca_solver=0, inner_reduction=0.0, j_lanes=0, ca_reduction=0.0, sweep_format=0,
                 single_stream=False, sweep_chunk=0, sweep_chain=True, j_slabs=0, sweep_fuse=False,
                 autotune=False, sweep_lanes=0, variant="PT", time_parallel=0, time_coarse_degree=0):
        self._ub = np.ascontiguousarray(ubar, dtype=np.float64)
        self._ab = np.ascontiguousarray(abar, dtype=np.float64)
        assert self._ub.shape == (nt, 2, (2 * n + 1) ** 2) and self._ab.shape == (nt, (n + 1) ** 2)
        self._jb = None if jbar is None else np.ascontiguousarray(jbar, dtype=np.float64)
        p = StProblem()
        p.n, p.nt, p.dt, p.mu, p.eta, p.mu0 = n, nt, dt, mu, eta, mu0
        p.ubar, p.abar = _dptr(self._ub), _dptr(self._ab)
        p.jbar = _dptr(self._jb) if self._jb is not None else ctypes.POINTER(ctypes.c_double)()
        p.precond_precision = ST_FP32 if precision == "fp32" else ST_FP64
        p.inner_mode = ST_INNER_EXACT if inner == "exact" else ST_INNER_AMG
        p.inner_iters, p.mass_iters, p.cheb_degree = inner_iters, mass_iters, cheb_degree
        p.max_restart, p.sell_sigma, p.adjoint = max_restart, sell_sigma, int(adjoint)
        p.fu_solver, p.ca_solver, p.inner_reduction, p.j_lanes = fu_solver, ca_solver, inner_reduction, j_lanes
        p.ca_reduction, p.sweep_format, p.single_stream = ca_reduction, sweep_format, int(single_stream)
        p.sweep_chunk = sweep_chunk
        p.sweep_chain = 0 if sweep_chain else -1
        p.j_slabs = j_slabs
        p.sweep_fuse = 1 if sweep_fuse else 0
        p.autotune = int(autotune)
        p.sweep_lanes = sweep_lanes
        p.precond_variant = {"PT": 0, "Ptilde": 1, "P": 2}[variant]
        p.time_parallel, p.time_coarse_degree = time_parallel, time_coarse_degree
        self.problem = p
        self.n, self.nt = n, nt
        h = ctypes.c_void_p()
        _check(lib().st_plan_create(ctypes.byref(p), ctypes.byref(h)), "st_plan_create")
        self.ptr = h
        ns = ctypes.c_int()
        offs = (ctypes.c_int * 6)()
        _check(lib().st_plan_sizes(self.ptr, ctypes.byref(ns), offs), "st_plan_sizes")
        self.ns = ns.value
        self.offsets = list(offs)
        wb = ctypes.c_size_t()
        _check(lib().st_plan_workspace_size(self.ptr, ctypes.byref(wb)), "st_plan_workspace_size")
        self.workspace_bytes = wb.value

    def export_block(self, name, k=0):
        """CSR (scipy) of a host-assembled block for slab k."""
        import scipy.sparse as sp
        bid = BLOCK_IDS[name]
        nr, nc, nnz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        ip = ctypes.POINTER(ctypes.c_int)
        _check(lib().st_plan_export_block(self.ptr, bid, k, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nnz),
                                          ip(), ip(), ctypes.POINTER(ctypes.c_double)()), "export")
        rp = np.empty(nr.value + 1, dtype=np.int32)
        ci = np.empty(nnz.value, dtype=np.int32)
        v = np.empty(nnz.value, dtype=np.float64)
        _check(lib().st_plan_export_block(self.ptr, bid, k, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nnz),
                                          rp.ctypes.data_as(ip), ci.ctypes.data_as(ip), _dptr(v)), "export")
        return sp.csr_matrix((v, ci, rp), shape=(nr.value, nc.value))

    def block_nnz(self, name, k=0):
        nr, nc, nnz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        ip = ctypes.POINTER(ctypes.c_int)
        _check(lib().st_plan_export_block(self.ptr, BLOCK_IDS[name], k, ctypes.byref(nr), ctypes.byref(nc),
                                          ctypes.byref(nnz), ip(), ip(), ctypes.POINTER(ctypes.c_double)()), "nnz")
        return nnz.value

    def cheb_intervals(self, which):
        """(nt, 2) array of the (theta, delta) Chebyshev-alone intervals of F_u,k
        ("Fu") or C_A,k ("CA") per slab."""
        out = np.zeros((self.nt, 2))
        _check(lib().st_plan_cheb_intervals(self.ptr, {"Fu": 0, "CA": 1}[which], _dptr(out)), "cheb_intervals")
        return out

    def solver_info(self):
        """(fu_degree, ca_degree, fu_kappa, ca_kappa) chosen by the setup (degree 0 = AMG)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        c, d = ctypes.c_double(), ctypes.c_double()
        _check(lib().st_plan_solver_info(self.ptr, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                         ctypes.byref(d)), "solver_info")
        return a.value, b.value, c.value, d.value

    def jacobian_slots(self):
        """([per-slab, slab-invariant, coupling] SELL entries of J with padding, slices)."""
        slots = (ctypes.c_int64 * 3)()
        ns = ctypes.c_int()
        _check(lib().st_plan_jacobian_slots(self.ptr, slots, ctypes.byref(ns)), "jacobian_slots")
        return list(slots), ns.value

    def export_jbar(self):
        out = np.empty((self.nt, (self.n + 1) ** 2))
        _check(lib().st_plan_export_jbar(self.ptr, _dptr(out)), "export_jbar")
        return out

    def close(self):
        if self.ptr:
            lib().st_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class System:
    """A device-resident space-time system (``st_create``) with torch-owned memory."""

    def __init__(self, plan: Plan, device="cuda:0", stream=None):
        import torch
        self.device = torch.device(device)
        self.ws = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        h = ctypes.c_void_p()
        _check(lib().st_create(plan.ptr, ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(plan.workspace_bytes),
                               _stream_ptr(stream), ctypes.byref(h)), "st_create")
        self.ptr = h
        self.ns, self.nt, self.n = plan.ns, plan.nt, plan.n
        self.N = self.ns * self.nt
        self.offsets = plan.offsets

    def _vec(self, t):
        import torch
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and t.numel() == self.N
        return ctypes.c_void_p(t.data_ptr())

    def apply_jacobian(self, x, y=None, transpose=False, stream=None):
        import torch
        y = torch.empty_like(x) if y is None else y
        fn = lib().st_apply_jacobian_t if transpose else lib().st_apply_jacobian
        _check(fn(self.ptr, self._vec(x), self._vec(y), _stream_ptr(stream)), "st_apply_jacobian")
        return y

    def apply_precond(self, r, z=None, transpose=False, stream=None):
        import torch
        z = torch.empty_like(r) if z is None else z
        fn = lib().st_apply_precond_t if transpose else lib().st_apply_precond
        _check(fn(self.ptr, self._vec(r), self._vec(z), _stream_ptr(stream)), "st_apply_precond")
        return z

    def apply_precond_noalloc(self, r, z, stream=None):
        """z = P_T^{-1} r with the library's static scratch (``st_apply_precond_noalloc``):
        no device allocation in the call; z must be given."""
        _check(lib().st_apply_precond_noalloc(self.ptr, self._vec(r), self._vec(z), _stream_ptr(stream)),
               "st_apply_precond_noalloc")
        return z

    def initial_coupling(self, a0, y=None, stream=None):
        """y = (M_A / dt) a0 on the interior potential nodes (FP64, device)."""
        import torch
        na = self.offsets[5] - self.offsets[4]
        assert a0.dtype == torch.float64 and a0.is_cuda and a0.is_contiguous() and a0.numel() == na
        y = torch.empty_like(a0) if y is None else y
        _check(lib().st_apply_initial_coupling(self.ptr, ctypes.c_void_p(a0.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                               _stream_ptr(stream)), "st_apply_initial_coupling")
        return y

    def solve(self, b, x=None, restart=30, rtol=1e-8, atol=0.0, maxit=1000, x0=False, history=0,
              adjoint=False, stream=None, orth="auto"):
        """FGMRES on J x = b (or the adjoint J^T x = b).  Returns (x, info, status, history).
        ``orth``: Gram-Schmidt of the Arnoldi steps, "auto", "cgs2" or "delayed" (``st_opts.orth``;
        automatic: delayed reorthogonalisation above restart 64 or from 2^20 unknowns)."""
        import torch
        x = torch.zeros_like(b) if x is None else x
        o = StOpts()
        o.restart, o.maxit, o.rtol, o.atol, o.x0_given = restart, maxit, rtol, atol, int(x0)
        o.orth = ORTH[orth]
        hist = np.zeros(max(history, 0))
        o.history_len = hist.size
        o.history = _dptr(hist) if hist.size else ctypes.POINTER(ctypes.c_double)()
        info = StInfo()
        fn = lib().st_adjoint_solve if adjoint else lib().st_fgmres_solve
        rc = _check(fn(self.ptr, self._vec(b), self._vec(x), ctypes.byref(o), ctypes.byref(info),
                       _stream_ptr(stream)), "solve")
        return x, info, rc, hist[:min(info.iterations + 1, hist.size)]

    def tuning(self):
        """Launch choices in effect (``st_tuning``): J slabs per wavefront, sweep
        step rows per workgroup, tiled sweep solves, launches per P_T apply."""
        js, rows, fuse, pl, lanes = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().st_tuning(self.ptr, ctypes.byref(js), ctypes.byref(rows), ctypes.byref(fuse), ctypes.byref(pl),
                               ctypes.byref(lanes)), "st_tuning")
        return {"j_slabs": js.value, "step_rows": rows.value, "sweep_fuse": bool(fuse.value),
                "precond_launches": pl.value, "step_lanes": lanes.value}

    def profile_kernel(self, kernel=1, every=8):
        """Sampled event timing of the paired sweep-step kernel (``st_profile_kernel``)."""
        _check(lib().st_profile_kernel(self.ptr, kernel, every), "st_profile_kernel")

    def profile_read(self):
        """(seconds summed over timed launches, launches timed, launches seen)."""
        sec, n, seen = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().st_profile_read(self.ptr, ctypes.byref(sec), ctypes.byref(n), ctypes.byref(seen)),
               "st_profile_read")
        return sec.value, n.value, seen.value

    def close(self):
        if getattr(self, "ptr", None):
            lib().st_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TimeStepping:
    """Sequential time stepping with the single-step preconditioner P_{T,k}
    (``st_timestep_solve``): one one-slab system per slab of the state; with
    ``window`` W > 1, windows of W slabs (the last one shorter), each solved all
    at once with its own P_T (windowed space-time)."""

    def __init__(self, n, nt, dt, mu, eta, mu0, ubar, abar, device="cuda:0", precision="fp64", inner="amg",
                 restart=30, window=1, **plan_kw):
        if int(window) < 1:
            raise ValueError(f"window must be at least 1 slab, got {window}")
        self.systems = []
        for k0 in range(0, nt, window):
            w = min(window, nt - k0)
            plan = Plan(n, w, dt, mu, eta, mu0, ubar[k0:k0 + w], abar[k0:k0 + w], precision=precision,
                        inner=inner, max_restart=restart, **plan_kw)
            self.systems.append(System(plan, device))
            plan.close()
        self.nt, self.ns, self.restart, self.window = nt, self.systems[0].ns, restart, window
        self.N = self.nt * self.ns
        self.offsets = self.systems[0].offsets

    def solve(self, b, x=None, rtol=1e-8, atol=0.0, maxit=1000, warm_start=True, stream=None):
        """Returns (x, per-step (per-window) infos, status)."""
        import torch
        assert b.dtype == torch.float64 and b.is_cuda and b.is_contiguous() and b.numel() == self.N
        x = torch.zeros_like(b) if x is None else x
        o = StOpts()
        o.restart, o.maxit, o.rtol, o.atol, o.x0_given = self.restart, maxit, rtol, atol, int(warm_start)
        o.history_len = 0
        o.history = ctypes.POINTER(ctypes.c_double)()
        nw = len(self.systems)
        infos = (StInfo * nw)()
        arr = (ctypes.c_void_p * nw)(*[s.ptr.value for s in self.systems])
        rc = _check(lib().st_timestep_solve(arr, nw, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                            ctypes.byref(o), infos, _stream_ptr(stream)), "st_timestep_solve")
        return x, list(infos), rc


class Newton:
    """Space-time Newton on the nonlinear recurrence (``st_nl_*``, ``st_newton_solve``).

    ``fields`` holds host arrays u_base, p_base, a_base, u_init, a_init and
    optionally j_base, f, e (see ``st_nl_problem``).  Without j_base the base
    current is the one a plan computes from the base potential (its discrete
    current equation, ``st_plan_export_jbar``).  ``plan_kw`` are the options of
    every linearisation's plan (precision, inner solvers, ...)."""

    def __init__(self, n, nt, dt, mu, eta, mu0, fields, device="cuda:0", stream=None, **plan_kw):
        import torch
        self.n, self.nt, self.dt, self.mu, self.eta, self.mu0 = n, nt, dt, mu, eta, mu0
        arr = {k: (None if v is None else np.ascontiguousarray(v, dtype=np.float64)) for k, v in fields.items()}
        # the plan of the base state: template of every linearisation, and the base current
        plan = Plan(n, nt, dt, mu, eta, mu0, arr["u_base"], arr["a_base"], jbar=arr.get("j_base"), **plan_kw)
        if arr.get("j_base") is None:
            arr["j_base"] = plan.export_jbar()
        self.template = plan.problem
        self.template.ubar = self.template.abar = self.template.jbar = ctypes.POINTER(ctypes.c_double)()
        self.lin_bytes = plan.workspace_bytes
        plan.close()
        self._arr = arr
        p = StNlProblem()
        p.n, p.nt, p.dt, p.mu, p.eta, p.mu0 = n, nt, dt, mu, eta, mu0
        null = ctypes.POINTER(ctypes.c_double)()
        for k in ("u_base", "p_base", "j_base", "a_base", "u_init", "a_init", "f", "e"):
            setattr(p, k, _dptr(arr[k]) if arr.get(k) is not None else null)
        self.problem = p
        wb = ctypes.c_size_t()
        _check(lib().st_nl_workspace_size(ctypes.byref(p), ctypes.byref(wb)), "st_nl_workspace_size")
        self.device = torch.device(device)
        self.ws = torch.empty(wb.value + 256, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(lib().st_nl_create(ctypes.byref(p), ctypes.c_void_p((self.ws.data_ptr() + 255) & ~255),
                                  ctypes.c_size_t(wb.value), _stream_ptr(stream), ctypes.byref(h)), "st_nl_create")
        self.ptr = h
        self.ns = int(inputs_slab_size(n))
        self.N = self.ns * nt
        # the linear workspace, reused by every linearisation (a quarter of margin for
        # hierarchies whose sizes follow the state)
        self.lin_ws_bytes = int(self.lin_bytes * 1.25) + (1 << 20)
        self.lin_ws = torch.empty(self.lin_ws_bytes + 256, dtype=torch.uint8, device=self.device)

    def residual(self, x, r=None, stream=None):
        import torch
        r = torch.empty_like(x) if r is None else r
        _check(lib().st_nl_residual(self.ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                    _stream_ptr(stream)), "st_nl_residual")
        return r

    def solve(self, x=None, atol=1e-10, max_newton=20, lin_rtol=1e-2, lin_atol=1e-14, restart=30, maxit=1000,
              stream=None):
        """Newton from x (zero if None), updated in place.  Returns (x, info, status)."""
        import torch
        x = torch.zeros(self.N, dtype=torch.float64, device=self.device) if x is None else x
        o = StNewtonOpts()
        o.max_newton, o.atol = max_newton, atol
        o.linear.restart, o.linear.maxit, o.linear.rtol, o.linear.atol = restart, maxit, lin_rtol, lin_atol
        o.linear.history_len = 0
        o.linear.history = ctypes.POINTER(ctypes.c_double)()
        info = StNewtonInfo()
        ws_ptr = (self.lin_ws.data_ptr() + 255) & ~255
        rc = _check(lib().st_newton_solve(self.ptr, ctypes.byref(self.template), ctypes.c_void_p(ws_ptr),
                                          ctypes.c_size_t(self.lin_ws_bytes), ctypes.c_void_p(x.data_ptr()),
                                          ctypes.byref(o), ctypes.byref(info), _stream_ptr(stream)),
                    "st_newton_solve")
        return x, info, rc

    def close(self):
        if getattr(self, "ptr", None):
            lib().st_nl_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def inputs_slab_size(n):
    """Unknowns of one slab: interior u (2 components), all p and j, interior A."""
    return 2 * (2 * n - 1) ** 2 + 2 * (n + 1) ** 2 + (n - 1) ** 2


class Batch:
    """Lockstep FGMRES over several systems (``st_batch_*``, ``st_fgmres_solve_batched``).

    The systems must share the preconditioner precision and stay alive while
    the batch exists; the batch's own device memory (the recorded launches) is
    a torch tensor.
    """

    def __init__(self, systems, restart=30, stream=None):
        import torch
        self.systems = list(systems)
        n = len(self.systems)
        arr = (ctypes.c_void_p * n)(*[s.ptr.value for s in self.systems])
        h = ctypes.c_void_p()
        _check(lib().st_batch_create(arr, n, restart, ctypes.byref(h)), "st_batch_create")
        self.ptr = h
        self.restart = restart
        wb = ctypes.c_size_t()
        _check(lib().st_batch_workspace_size(self.ptr, ctypes.byref(wb)), "st_batch_workspace_size")
        self.workspace_bytes = wb.value
        dev = self.systems[0].device
        self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        self._ws_ptr = (self.ws.data_ptr() + 255) & ~255
        _check(lib().st_batch_upload(self.ptr, ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(self.workspace_bytes),
                                     _stream_ptr(stream)), "st_batch_upload")

    def launch_counts(self):
        """(lockstep, separate) launches of one Arnoldi step over the batch."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().st_batch_launch_counts(self.ptr, ctypes.byref(a), ctypes.byref(b)), "launch_counts")
        return a.value, b.value

    def solve(self, bs, xs=None, rtol=1e-8, atol=0.0, maxit=1000, x0=False, history=0, stream=None,
              orth="auto"):
        """Solves every member; returns (xs, infos, statuses, rc, histories).  The
        lockstep steps use CGS2 ("auto" or "cgs2"; "delayed" is rejected)."""
        import torch
        n = len(self.systems)
        assert len(bs) == n
        xs = [torch.zeros_like(b) for b in bs] if xs is None else xs
        for s, b, x in zip(self.systems, bs, xs):
            s._vec(b)
            s._vec(x)
        barr = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
        xarr = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        o = StOpts()
        o.restart, o.maxit, o.rtol, o.atol, o.x0_given = self.restart, maxit, rtol, atol, int(x0)
        o.orth = ORTH[orth]
        hist = np.zeros((n, max(history, 0)))
        o.history_len = hist.shape[1]
        o.history = _dptr(hist) if hist.size else ctypes.POINTER(ctypes.c_double)()
        infos = (StInfo * n)()
        st = (ctypes.c_int * n)()
        rc = _check(lib().st_fgmres_solve_batched(self.ptr, barr, xarr, ctypes.byref(o), infos, st,
                                                  _stream_ptr(stream)), "st_fgmres_solve_batched")
        return xs, list(infos), list(st), rc, hist

    def close(self):
        if getattr(self, "ptr", None):
            lib().st_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
