"""Python binding of libfg (ctypes).  Argument marshalling only: every step of
the solver runs in libfg's HIP kernels; torch supplies device memory and the
stream.  Raises when the library or the GPU is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfg.so")

FG_OK, FG_NOT_CONVERGED = 0, 1
FG_ERR_ARG, FG_ERR_OOM, FG_ERR_BREAKDOWN, FG_ERR_NAN, FG_ERR_HIP, FG_ERR_STATE = -1, -2, -3, -4, -5, -6
FG_K, FG_A22, FG_KBULK, FG_C, FG_K_EXACT = 0, 1, 2, 3, 4
FG_F64, FG_F32, FG_MIXED, FG_MIXED_F32VAL = 0, 1, 2, 3

SYMBOLS = ["fg_last_error", "fg_ctx_create", "fg_ctx_destroy", "fg_system_create", "fg_system_destroy",
           "fg_assemble", "fg_cohesive_update", "fg_pcg_solve", "fg_flow_solve", "fg_step", "fg_spmv",
           "fg_coupling", "fg_residual", "fg_system_sizes", "fg_export", "fg_profile", "fg_profile_read", "fg_tune", "fg_adjoint_solve", "fg_group_stats",
           "fg_assemble_groups", "fg_slip_adjoint", "fg_cheb_interval", "fg_exact_solve", "fg_adjoint_loop_step", "fg_pcg_solve_noalloc",
           "fg_lanczos_bounds", "fg_amg_levels", "fg_amg_aggregates"]


class FgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libfg status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("nu", "alpha", "biot_M", "mu", "k_par", "k_perp", "w0", "M_F", "k_n", "k_s", "friction", "dt")]


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_tets", C.c_int64), ("n_coh", C.c_int64),
                ("xyz_h", C.c_void_p), ("tets_h", C.c_void_p), ("coh_h", C.c_void_p),
                ("dir_u_h", C.c_void_p), ("dir_p_h", C.c_void_p), ("group_h", C.c_void_p)]


class PcgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("precision", C.c_int),
                ("check_every", C.c_int), ("inner_tol", C.c_double)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("cycles", C.c_int64), ("relres", C.c_double), ("status", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("newton_iters", C.c_int64), ("outer_iters", C.c_int64), ("inner_k_iters", C.c_int64),
                ("inner_a22_iters", C.c_int64), ("outer_relres", C.c_double), ("res_m", C.c_double),
                ("res_f", C.c_double), ("status", C.c_int), ("step_cuts", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libfg.so (built by __graft_entry__.build / paper_2410_17133_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FgError(FG_ERR_STATE, f"{LIB_PATH} is missing: build it first (python __graft_entry__.py)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
        L.fg_last_error.restype = C.c_char_p
        sig = {
            "fg_ctx_create": [C.POINTER(vp), i32],
            "fg_ctx_destroy": [vp],
            "fg_system_create": [vp, C.POINTER(Mesh), C.POINTER(vp)],
            "fg_system_destroy": [vp],
            "fg_assemble": [vp, vp, C.POINTER(Params), vp, vp, vp],
            "fg_assemble_groups": [vp, vp, C.POINTER(Params), i32, vp, vp, vp],
            "fg_cohesive_update": [vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp],
            "fg_pcg_solve": [vp, vp, i32, i32, vp, vp, C.POINTER(PcgOpts), C.POINTER(PcgInfo), vp],
            "fg_flow_solve": [vp, vp, vp, vp, vp, vp, C.POINTER(PcgOpts), C.POINTER(PcgOpts), dbl, i64,
                              C.POINTER(SolveInfo), vp],
            "fg_step": [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, dbl, i64, C.POINTER(PcgOpts), C.POINTER(PcgOpts),
                        dbl, i64, C.POINTER(SolveInfo), vp],
            "fg_spmv": [vp, vp, i32, vp, vp, vp],
            "fg_coupling": [vp, vp, i32, vp, vp, vp],
            "fg_residual": [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
            "fg_system_sizes": [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)],
            "fg_export": [vp, vp, i32, vp, vp, vp, vp],
            "fg_profile": [vp, i32],
            "fg_tune": [vp, C.c_char_p, i64],
            "fg_group_stats": [vp, vp, vp, vp, C.POINTER(i32)],
            "fg_adjoint_solve": [vp, vp] + [vp] * 11 + [C.POINTER(PcgOpts), C.POINTER(PcgOpts), dbl, dbl, i64,
                                                        C.POINTER(SolveInfo), vp],
            "fg_profile_read": [vp, i32, C.POINTER(i64), C.POINTER(dbl), i32],
            "fg_slip_adjoint": [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
            "fg_cheb_interval": [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double), vp],
            "fg_exact_solve": [vp, vp, vp, vp, C.POINTER(PcgOpts), C.POINTER(PcgInfo), vp],
            "fg_amg_levels": [vp, vp, C.POINTER(C.c_int), vp, vp],
            "fg_amg_aggregates": [vp, vp, i32, vp, vp],
            "fg_lanczos_bounds": [vp, vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double), vp],
            "fg_pcg_solve_noalloc": [vp, vp, i32, vp, vp, C.POINTER(PcgOpts), C.POINTER(PcgInfo), vp],
            "fg_adjoint_loop_step": [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                     C.POINTER(PcgOpts), C.POINTER(PcgOpts), dbl, dbl, i64, C.POINTER(SolveInfo), vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, allow_not_converged=True):
    if status == FG_OK or (status == FG_NOT_CONVERGED and allow_not_converged):
        return status
    raise FgError(status, lib().fg_last_error().decode())


def _ptr(t, dtype, n=None, name="tensor"):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise FgError(FG_ERR_ARG, f"{name}: expected a contiguous {dtype} CUDA tensor")
    if n is not None and t.numel() != n:
        raise FgError(FG_ERR_ARG, f"{name}: expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def opts(tol=1e-10, max_iter=1000000, precision=FG_F64, check_every=32, inner_tol=0.0):
    """Solver options; inner_tol 0 takes the library's default for the precision."""
    return PcgOpts(tol, max_iter, precision, check_every, inner_tol)


class Context:
    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise FgError(FG_ERR_STATE, "no HIP device visible")
        h = C.c_void_p()
        _check(lib().fg_ctx_create(C.byref(h), device))
        self._h = h
        self.device = torch.device("cuda", device)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fg_ctx_destroy(self._h)
            self._h = None


class System:
    """A planned mesh with its assembled operators on the GPU."""

    def __init__(self, ctx: Context, xyz, tets, coh, dir_u, dir_p, group=None):
        self.ctx = ctx
        self._keep = [np.ascontiguousarray(xyz, np.float64), np.ascontiguousarray(tets, np.int32),
                      np.ascontiguousarray(coh if len(coh) else np.zeros((0, 6)), np.int32),
                      np.ascontiguousarray(dir_u, np.uint8), np.ascontiguousarray(dir_p, np.uint8),
                      None if group is None else np.ascontiguousarray(group, np.int32)]
        x, t, c, du, dp, gr = self._keep
        self.ngroups = 1 if gr is None else int(gr.max()) + 1
        self.N, self.ne, self.nf = x.shape[0], t.shape[0], c.shape[0]
        self.nq = 3 * self.nf
        m = Mesh(self.N, self.ne, self.nf, x.ctypes.data, t.ctypes.data, c.ctypes.data if self.nf else None,
                 du.ctypes.data, dp.ctypes.data, None if gr is None else gr.ctypes.data)
        h = C.c_void_p()
        _check(lib().fg_system_create(ctx._h, C.byref(m), C.byref(h)))
        self._h = h
        self.dev = ctx.device

    @classmethod
    def from_instance(cls, ctx, inst):
        m = inst.mesh
        return cls(ctx, m.xyz, m.tets, m.coh, inst.dir_u, inst.dir_p)

    @classmethod
    def from_batch(cls, ctx, batch):
        """A batch of independent instances (inputs.concat_instances) as one grouped system."""
        return cls(ctx, batch.xyz, batch.tets, batch.coh, batch.dir_u, batch.dir_p, batch.group)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fg_system_destroy(self._h)
            self._h = None

    def sizes(self):
        """(stored blocks, padded blocks, slices, total halo entries)."""
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().fg_system_sizes(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return a.value, b.value, c.value, d.value

    def _d(self, n, dtype=torch.float64):
        return torch.zeros(n, dtype=dtype, device=self.dev)

    def assemble(self, params, E, logk):
        """params: one parameter set, or a list with one per group of a batch system."""
        many = isinstance(params, (list, tuple))
        conv = lambda p: Params(*p.as_tuple()) if hasattr(p, "as_tuple") else p
        plist = [conv(p) for p in params] if many else [conv(params)]
        arr = (Params * len(plist))(*plist)
        self.params = plist[0]
        self.E = E if isinstance(E, torch.Tensor) else torch.as_tensor(np.asarray(E, np.float64), device=self.dev)
        self.logk = logk if isinstance(logk, torch.Tensor) else torch.as_tensor(np.asarray(logk, np.float64), device=self.dev)
        _check(lib().fg_assemble_groups(self.ctx._h, self._h, arr, len(plist),
                                        _ptr(self.E, torch.float64, self.ne, "E"),
                                        _ptr(self.logk, torch.float64, self.ne, "log_k"), _stream()))

    def cohesive_update(self, U, die_n, t0, write_tangent=True):
        nq = self.nq
        trac, die = self._d(3 * nq), self._d(2 * nq)
        flag = self._d(nq, torch.uint8)
        fcoh = self._d(3 * self.N)
        _check(lib().fg_cohesive_update(self.ctx._h, self._h, _ptr(U, torch.float64, 3 * self.N, "U"),
                                        _ptr(die_n, torch.float64, 2 * nq, "die_n"), _ptr(t0, torch.float64, 3 * nq, "t0"),
                                        _ptr(trac, torch.float64), _ptr(die, torch.float64), _ptr(flag, torch.uint8),
                                        _ptr(fcoh, torch.float64), int(bool(write_tangent)), _stream()))
        return trac, die, flag, fcoh

    def pcg_solve(self, which, b, nrhs=1, **kw):
        n = (3 if which == FG_K else 1) * self.N * nrhs
        x = self._d(n)
        info = PcgInfo()
        st = lib().fg_pcg_solve(self.ctx._h, self._h, which, nrhs, _ptr(b, torch.float64, n, "b"),
                                _ptr(x, torch.float64), C.byref(opts(**kw)), C.byref(info), _stream())
        _check(st)
        return x, info

    def pcg_solve_noalloc(self, which, b, x, **kw):
        """fg_pcg_solve_noalloc: one right-hand side, the solution written into the caller's x
        (the call allocates no device memory; x must be a CUDA float64 tensor).  Returns info."""
        n = (3 if which == FG_K else 1) * self.N
        info = PcgInfo()
        st = lib().fg_pcg_solve_noalloc(self.ctx._h, self._h, which, _ptr(b, torch.float64, n, "b"),
                                        _ptr(x, torch.float64, n, "x"), C.byref(opts(**kw)), C.byref(info), _stream())
        _check(st)
        return info

    def exact_solve(self, b, **kw):
        """(K_t + N) x = b by BiCGStab (fg_exact_solve): the exact interface tangent of the last
        interface update.  Returns (x, info)."""
        n = 3 * self.N
        x = self._d(n)
        info = PcgInfo()
        st = lib().fg_exact_solve(self.ctx._h, self._h, _ptr(b, torch.float64, n, "b"), _ptr(x, torch.float64),
                                  C.byref(opts(**kw)), C.byref(info), _stream())
        _check(st)
        return x, info

    def flow_solve(self, b_u, b_p, inner_k=None, inner_p=None, outer_tol=1e-10, outer_max_iter=1000):
        du, dp = self._d(3 * self.N), self._d(self.N)
        info = SolveInfo()
        ik = inner_k or opts(tol=1e-12)
        ip = inner_p or opts(tol=1e-12)
        st = lib().fg_flow_solve(self.ctx._h, self._h, _ptr(b_u, torch.float64, 3 * self.N, "b_u"),
                                 _ptr(b_p, torch.float64, self.N, "b_p"), _ptr(du, torch.float64),
                                 _ptr(dp, torch.float64), C.byref(ik), C.byref(ip), outer_tol, outer_max_iter,
                                 C.byref(info), _stream())
        _check(st)
        return du, dp, info

    def step(self, U, P, die, t0, F_u, f_p, newton_tol=1e-10, newton_max_iter=30, inner_k=None, inner_p=None,
             outer_tol=1e-10, outer_max_iter=1000):
        """One implicit step; U, P, die (CUDA float64) are updated in place."""
        nq = self.nq
        trac = self._d(3 * nq)
        flag = self._d(nq, torch.uint8)
        info = SolveInfo()
        ik = inner_k or opts(tol=1e-12)
        ip = inner_p or opts(tol=1e-12)
        st = lib().fg_step(self.ctx._h, self._h, _ptr(U, torch.float64, 3 * self.N, "U"),
                           _ptr(P, torch.float64, self.N, "P"), _ptr(die, torch.float64, 2 * nq, "die"),
                           _ptr(trac, torch.float64), _ptr(flag, torch.uint8), _ptr(t0, torch.float64, 3 * nq, "t0"),
                           _ptr(F_u, torch.float64, 3 * self.N, "F_u"), _ptr(f_p, torch.float64, self.N, "f_p"),
                           newton_tol, newton_max_iter, C.byref(ik), C.byref(ip), outer_tol, outer_max_iter,
                           C.byref(info), _stream())
        _check(st)
        return trac, flag, info

    def adjoint(self, U, P, die_n, t0, logk, dJdU, dJdP, inner_k=None, inner_p=None, outer_tol=1e-12,
                defect_tol=1e-12, max_defect_iters=50, multipliers=False):
        """Gradient of J w.r.t. (E, ln k) at a converged step state: returns (dJ_dE, dJ_dlogk, info)
        or, with multipliers=True, (dJ_dE, dJ_dlogk, lam_u, lam_p, info)."""
        dE, dk = self._d(self.ne), self._d(self.ne)
        lu = self._d(3 * self.N) if multipliers else None
        lp = self._d(self.N) if multipliers else None
        info = SolveInfo()
        ik = inner_k or opts(tol=1e-13)
        ip = inner_p or opts(tol=1e-13)
        nq = self.nq
        st = lib().fg_adjoint_solve(self.ctx._h, self._h, _ptr(U, torch.float64, 3 * self.N, "U"),
                                    _ptr(P, torch.float64, self.N, "P"), _ptr(die_n, torch.float64, 2 * nq, "die_n"),
                                    _ptr(t0, torch.float64, 3 * nq, "t0"), _ptr(logk, torch.float64, self.ne, "log_k"),
                                    _ptr(dJdU, torch.float64, 3 * self.N, "dJdU"), _ptr(dJdP, torch.float64, self.N, "dJdP"),
                                    _ptr(dE, torch.float64), _ptr(dk, torch.float64), _ptr(lu, torch.float64),
                                    _ptr(lp, torch.float64), C.byref(ik), C.byref(ip), outer_tol, defect_tol,
                                    max_defect_iters, C.byref(info), _stream())
        _check(st)
        if multipliers:
            return dE, dk, lu, lp, info
        return dE, dk, info

    def adjoint_loop_step(self, U, P, die_old, t0, logk, dJdU, dJdP, lam_p_next, a, dJ_dE, dJ_dlogk, lam_p,
                          inner_k=None, inner_p=None, outer_tol=1e-12, defect_tol=1e-12, max_defect_iters=50):
        """One step of the reverse sweep through a time loop (fg_adjoint_loop_step): a [nq*2]
        is updated in place (a_n in, a_{n-1} out), dJ_dE and dJ_dlogk are accumulated, and
        lam_p receives the step's pressure multipliers (lam_p_next of the next call)."""
        info = SolveInfo()
        ik = inner_k or opts(tol=1e-13)
        ip = inner_p or opts(tol=1e-13)
        nq, N = self.nq, self.N
        st = lib().fg_adjoint_loop_step(
            self.ctx._h, self._h, _ptr(U, torch.float64, 3 * N, "U"), _ptr(P, torch.float64, N, "P"),
            _ptr(die_old, torch.float64, 2 * nq, "die_old"), _ptr(t0, torch.float64, 3 * nq, "t0"),
            _ptr(logk, torch.float64, self.ne, "log_k"), _ptr(dJdU, torch.float64, 3 * N, "dJdU"),
            _ptr(dJdP, torch.float64, N, "dJdP"), _ptr(lam_p_next, torch.float64, N, "lam_p_next"),
            _ptr(a, torch.float64, 2 * nq, "a"), _ptr(dJ_dE, torch.float64, self.ne, "dJ_dE"),
            _ptr(dJ_dlogk, torch.float64, self.ne, "dJ_dlogk"), None, _ptr(lam_p, torch.float64, N, "lam_p"),
            C.byref(ik), C.byref(ip), outer_tol, defect_tol, max_defect_iters, C.byref(info), _stream())
        _check(st)
        return info

    def slip_adjoint(self, U, die_old, t0, a_new, lam_u=None):
        """(gU [3N], a_old [nq*2]) of the slip state carried between steps (fg_slip_adjoint)."""
        nq = self.nq
        gU, a_old = self._d(3 * self.N), self._d(2 * nq)
        _check(lib().fg_slip_adjoint(self.ctx._h, self._h, _ptr(U, torch.float64, 3 * self.N, "U"),
                                     _ptr(die_old, torch.float64, 2 * nq, "die_old"), _ptr(t0, torch.float64, 3 * nq, "t0"),
                                     _ptr(a_new, torch.float64, 2 * nq, "a_new"),
                                     None if lam_u is None else _ptr(lam_u, torch.float64, 3 * self.N, "lam_u"),
                                     _ptr(gU, torch.float64), _ptr(a_old, torch.float64), _stream()), False)
        return gU, a_old

    def amg_levels(self):
        """(levels, nodes per level) of the AMG hierarchy of k_precond 3 (fg_amg_levels)."""
        nl = C.c_int()
        nodes = np.zeros(6, np.int64)
        _check(lib().fg_amg_levels(self.ctx._h, self._h, C.byref(nl), nodes.ctypes.data, _stream()), False)
        return nl.value, nodes[:nl.value]

    def amg_aggregates(self, level):
        """Aggregate number of every node of AMG level `level` (fg_amg_aggregates; level 0 in
        the caller's node numbering), as a numpy int32 array."""
        nl, nodes = self.amg_levels()
        if not 0 <= level < nl - 1:
            raise ValueError(f"level must be in [0, {nl - 2}]")
        out = np.zeros(int(nodes[level]), np.int32)
        _check(lib().fg_amg_aggregates(self.ctx._h, self._h, int(level), out.ctypes.data, _stream()), False)
        return out

    def lanczos_bounds(self, steps):
        """(smallest, largest) Ritz values of `steps` block-Jacobi CG steps on the probe
        vector: estimates of the extreme eigenvalues of M^-1 K (fg_lanczos_bounds)."""
        lo, hi = C.c_double(), C.c_double()
        _check(lib().fg_lanczos_bounds(self.ctx._h, self._h, int(steps), C.byref(lo), C.byref(hi), _stream()), False)
        return lo.value, hi.value

    def cheb_interval(self):
        """(lo, hi) of the Chebyshev preconditioner of the current K (fg_cheb_interval)."""
        lo, hi = C.c_double(), C.c_double()
        _check(lib().fg_cheb_interval(self.ctx._h, self._h, C.byref(lo), C.byref(hi), _stream()), False)
        return lo.value, hi.value

    def spmv(self, which, x):
        n = (3 if which in (FG_K, FG_KBULK, FG_K_EXACT) else 1) * self.N
        y = self._d(n)
        _check(lib().fg_spmv(self.ctx._h, self._h, which, _ptr(x, torch.float64, n, "x"), _ptr(y, torch.float64),
                             _stream()), False)
        return y

    def coupling(self, x, transpose=False):
        nin, nout = (3 * self.N, self.N) if transpose else (self.N, 3 * self.N)
        y = self._d(nout)
        _check(lib().fg_coupling(self.ctx._h, self._h, int(transpose), _ptr(x, torch.float64, nin, "x"),
                                 _ptr(y, torch.float64), _stream()), False)
        return y

    def residual(self, U, P, U_n, P_n, f_coh, F_u, f_p):
        Rm, Rf = self._d(3 * self.N), self._d(self.N)
        n3, n1 = 3 * self.N, self.N
        _check(lib().fg_residual(self.ctx._h, self._h, _ptr(U, torch.float64, n3), _ptr(P, torch.float64, n1),
                                 _ptr(U_n, torch.float64, n3), _ptr(P_n, torch.float64, n1),
                                 _ptr(f_coh, torch.float64, n3), _ptr(F_u, torch.float64, n3),
                                 _ptr(f_p, torch.float64, n1), _ptr(Rm, torch.float64), _ptr(Rf, torch.float64),
                                 _stream()), False)
        return Rm, Rf

    def group_stats(self):
        """Per-group (iterations, relative residual, status) of the last solve on a batched system."""
        G = self.ngroups
        it, rr, stt = np.zeros(G, np.int64), np.zeros(G), np.zeros(G, np.int32)
        n = C.c_int()
        _check(lib().fg_group_stats(self._h, it.ctypes.data, rr.ctypes.data, stt.ctypes.data, C.byref(n)), False)
        return it, rr, stt

    def tune(self, key, value):
        _check(lib().fg_tune(self._h, key.encode(), int(value)), False)

    def profile(self, enable=True):
        _check(lib().fg_profile(self._h, int(bool(enable))), False)

    def profile_read(self, slot=0, reset=True):
        """(launches, milliseconds) of the timed CG product kernel for slot 0 = K FP64, 1 = K FP32, 2 = A22,
        3 = K with FP32 values and FP64 vectors."""
        n, ms = C.c_int64(), C.c_double()
        _check(lib().fg_profile_read(self._h, slot, C.byref(n), C.byref(ms), int(bool(reset))), False)
        return n.value, ms.value

    def export(self, which):
        """Assembled operator as node-pair blocks (rows, cols, vals), caller order, host numpy."""
        npairs = self.sizes()[0]
        bs = 9 if which in (FG_K, FG_KBULK) else 1
        rows, cols = np.zeros(npairs, np.int32), np.zeros(npairs, np.int32)
        vals = np.zeros(npairs * bs)
        _check(lib().fg_export(self.ctx._h, self._h, which, rows.ctypes.data, cols.ctypes.data, vals.ctypes.data,
                               _stream()), False)
        return rows, cols, vals.reshape(npairs, 3, 3) if bs == 9 else vals

    def scipy(self, which):
        """The exported operator as a scalar scipy CSR matrix (caller DOF order)."""
        import scipy.sparse as sp
        rows, cols, vals = self.export(which)
        if which in (FG_K, FG_KBULK):
            r = (3 * rows[:, None, None] + np.arange(3)[None, :, None]).repeat(3, 2).reshape(-1)
            c = (3 * cols[:, None, None] + np.arange(3)[None, None, :]).repeat(3, 1).reshape(-1)
            return sp.csr_matrix((vals.reshape(-1), (r, c)), shape=(3 * self.N, 3 * self.N))
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.N, self.N))
