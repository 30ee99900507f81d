"""ctypes wrapper of the CPU oracle (test infrastructure, not product code).

The oracle is a plain FP64 C reference of the solver's hot path (see the header
of oracle.c).  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")

K_BULK, K_TANGENT, A22, C_FLOW = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.c_int64, C.c_int64, C.c_int64, _f64p, _i32p, _i32p, _f64p, _f64p, _u8p, _u8p, _f64p]
        L.or_free.argtypes = [C.c_void_p]
        L.or_nnz.restype = C.c_int64
        L.or_nnz.argtypes = [C.c_void_p, C.c_int]
        L.or_get_csr.argtypes = [C.c_void_p, C.c_int, _i64p, _i32p, _f64p]
        L.or_spmv.argtypes = [C.c_void_p, C.c_int, _f64p, _f64p]
        L.or_cohesive.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, _f64p, _u8p, _f64p]
        L.or_apply_Apu.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_apply_Aup.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_pcg.restype = C.c_int
        L.or_pcg.argtypes = [C.c_void_p, C.c_int, _f64p, _f64p, C.c_double, C.c_int64,
                             C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.or_prevost.restype = C.c_int
        L.or_prevost.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, C.c_double, C.c_double, C.c_int64,
                                 C.c_int64, _f64p]
        L.or_residual.argtypes = [C.c_void_p] + [_f64p] * 9
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, _u8p, _f64p, _f64p, _f64p, C.c_double,
                              C.c_int64, C.c_double, C.c_double, C.c_int64, C.c_int64, C.c_int, _f64p]
        L.or_tet_grad.argtypes = [_f64p, C.POINTER(C.c_double), _f64p]
        L.or_tet_stiffness.argtypes = [_f64p, C.c_double, C.c_double, _f64p]
        L.or_tet_coupling.argtypes = [_f64p, C.c_double, _f64p]
        L.or_tet_flow.argtypes = [_f64p, C.c_double, C.c_double, _f64p, _f64p]
        L.or_tri_geom.argtypes = [_f64p, C.POINTER(C.c_double), _f64p, _f64p, _f64p, _f64p]
        L.or_tri_flow.argtypes = [_f64p, _f64p, _f64p, _f64p]
        L.or_return_map.restype = C.c_double
        L.or_return_map.argtypes = [_f64p, _f64p, _f64p, C.c_double, C.c_double, C.c_double, _f64p, _f64p, _u8p, _f64p]
        L.or_apply_NT.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_adjoint.restype = C.c_int
        L.or_adjoint.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, C.c_double, C.c_int64, C.c_double,
                                 C.c_double, C.c_int64, C.c_int64, _f64p]
        L.or_sensitivity.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.or_slip_adjoint.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_pcg_block.restype = C.c_int
        L.or_pcg_block.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int64, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]
        L.or_gj_inverse.argtypes = [C.c_int, _f64p, _f64p, C.POINTER(C.c_int)]
        L.or_cheb_apply.restype = C.c_int
        L.or_cheb_apply.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int, C.c_double, C.c_double]
        L.or_pcg_cheb.restype = C.c_int
        L.or_pcg_cheb.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int64, C.c_int, C.c_double, C.c_double,
                                  C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.or_probe_vector.argtypes = [C.c_void_p, _f64p]
        L.or_bj_lanczos.restype = C.c_int
        L.or_bj_lanczos.argtypes = [C.c_void_p, C.c_int, _f64p, _f64p]
        L.or_apply_N.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_bicgstab_exact.restype = C.c_int
        L.or_bicgstab_exact.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int64, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_double)]
        L.or_pcg_amg.restype = C.c_int
        L.or_pcg_amg.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int64, C.c_double, C.c_int64,
                                 C.POINTER(C.c_int64), C.POINTER(C.c_double), _f64p]
        L.or_amg_apply.restype = C.c_int
        L.or_amg_apply.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int64]
        L.or_amg_export.restype = C.c_int
        L.or_amg_export.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.c_int, C.c_int, _i64p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------- elements
def tet_grad(X):
    V = C.c_double()
    g = np.zeros(12)
    lib().or_tet_grad(_c(X, np.float64).reshape(-1), C.byref(V), g)
    return V.value, g.reshape(4, 3)


def tet_stiffness(X, E, nu):
    K = np.zeros(144)
    lib().or_tet_stiffness(_c(X, np.float64).reshape(-1), E, nu, K)
    return K.reshape(12, 12)


def tet_coupling(X, alpha):
    A = np.zeros(48)
    lib().or_tet_coupling(_c(X, np.float64).reshape(-1), alpha, A)
    return A.reshape(12, 4)


def tet_flow(X, k_over_mu, inv_M):
    S = np.zeros(16)
    Cm = np.zeros(16)
    lib().or_tet_flow(_c(X, np.float64).reshape(-1), k_over_mu, inv_M, S, Cm)
    return S.reshape(4, 4), Cm.reshape(4, 4)


def tri_geom(X):
    A = C.c_double()
    n, t1, t2, g = np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(9)
    lib().or_tri_geom(_c(X, np.float64).reshape(-1), C.byref(A), n, t1, t2, g)
    return A.value, n, t1, t2, g.reshape(3, 3)


def tri_flow(X, params):
    S = np.zeros(36)
    Cm = np.zeros(36)
    lib().or_tri_flow(_c(X, np.float64).reshape(-1), _c(params.as_tuple(), np.float64), S, Cm)
    return S.reshape(6, 6), Cm.reshape(6, 6)


def return_map(d, die_n, t0, kn, ks, f):
    trac, die, flag, D = np.zeros(3), np.zeros(2), np.zeros(1, np.uint8), np.zeros(9)
    nt = lib().or_return_map(_c(d, np.float64), _c(die_n, np.float64), _c(t0, np.float64), kn, ks, f,
                             trac, die, flag, D)
    return trac, die, int(flag[0]), D.reshape(3, 3), nt


# ---------------------------------------------------------------- problem
class Problem:
    """Assembled oracle system for one Instance (see paper_2410_17133_amd.inputs)."""

    def __init__(self, inst):
        m = inst.mesh
        self.inst = inst
        self.N = m.n_nodes
        self.nf = m.coh.shape[0]
        self.nq = 3 * self.nf
        L = lib()
        self._h = L.or_create(self.N, m.tets.shape[0], self.nf, _c(m.xyz, np.float64), _c(m.tets, np.int32),
                              _c(m.coh if self.nf else np.zeros((1, 6)), np.int32), _c(inst.E, np.float64),
                              _c(inst.logk, np.float64), _c(inst.dir_u, np.uint8), _c(inst.dir_p, np.uint8),
                              _c(inst.params.as_tuple(), np.float64))

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_free(self._h)
            self._h = None

    def csr(self, which):
        """(rowptr, col, val) of K_bulk / K tangent / A22 / C."""
        nnz = lib().or_nnz(self._h, which)
        n = 3 * self.N if which in (K_BULK, K_TANGENT) else self.N
        rp, col, val = np.zeros(n + 1, np.int64), np.zeros(nnz, np.int32), np.zeros(nnz)
        lib().or_get_csr(self._h, which, rp, col, val)
        return rp, col, val

    def scipy(self, which):
        import scipy.sparse as sp
        rp, col, val = self.csr(which)
        n = rp.size - 1
        return sp.csr_matrix((val, col, rp), shape=(n, n))

    def spmv(self, which, x):
        n = 3 * self.N if which in (K_BULK, K_TANGENT) else self.N
        y = np.zeros(n)
        lib().or_spmv(self._h, which, _c(x, np.float64), y)
        return y

    def cohesive(self, U, die_n, t0=None):
        t0 = self.inst.t0 if t0 is None else t0
        nq = max(self.nq, 1)
        trac, die, flag, f = np.zeros(nq * 3), np.zeros(nq * 2), np.zeros(nq, np.uint8), np.zeros(3 * self.N)
        lib().or_cohesive(self._h, _c(U, np.float64), _c(die_n, np.float64).reshape(-1),
                          _c(t0, np.float64).reshape(-1) if self.nq else np.zeros(3), trac, die, flag, f)
        return trac.reshape(-1, 3)[: self.nq], die.reshape(-1, 2)[: self.nq], flag[: self.nq], f

    def apply_Apu(self, p):
        out = np.zeros(3 * self.N)
        lib().or_apply_Apu(self._h, _c(p, np.float64), out)
        return out

    def apply_Aup(self, u):
        out = np.zeros(self.N)
        lib().or_apply_Aup(self._h, _c(u, np.float64), out)
        return out

    def pcg(self, which, b, tol=1e-10, maxit=100000):
        x = np.zeros_like(b, dtype=np.float64)
        it, rr = C.c_int64(), C.c_double()
        st = lib().or_pcg(self._h, which, _c(b, np.float64), x, tol, maxit, C.byref(it), C.byref(rr))
        return x, st, it.value, rr.value

    def pcg_block(self, b, tol=1e-10, maxit=1000000):
        """K_t x = b by PCG with the nodal / fault-pair block-Jacobi preconditioner: (x, status, iters, relres)."""
        x = np.zeros(3 * self.N)
        it, rr = C.c_int64(), C.c_double()
        st = lib().or_pcg_block(self._h, _c(b, np.float64), x, tol, maxit, C.byref(it), C.byref(rr))
        return x, st, it.value, rr.value

    def cheb_apply(self, r, degree, lo, hi):
        """z = p(M^-1 K_t) M^-1 r, the Chebyshev polynomial preconditioner over block Jacobi of
        the given degree on the spectrum interval [lo, hi] (Saad, Sec. 12.3)."""
        z = np.zeros(3 * self.N)
        st = lib().or_cheb_apply(self._h, _c(r, np.float64), z, int(degree), float(lo), float(hi))
        if st != 0:
            raise RuntimeError("a block of the block-Jacobi preconditioner is singular")
        return z

    def pcg_cheb(self, b, degree, lo, hi, tol=1e-10, maxit=1000000):
        """K_t x = b by PCG with the Chebyshev preconditioner: (x, status, iters, relres)."""
        x = np.zeros(3 * self.N)
        it, rr = C.c_int64(), C.c_double()
        st = lib().or_pcg_cheb(self._h, _c(b, np.float64), x, tol, maxit, int(degree), float(lo), float(hi),
                               C.byref(it), C.byref(rr))
        return x, st, it.value, rr.value

    def probe_vector(self):
        """SplitMix64 probe vector of the spectrum estimate (caller order, zero on Dirichlet DOFs)."""
        v = np.zeros(3 * self.N)
        lib().or_probe_vector(self._h, v)
        return v

    def bj_lanczos(self, steps):
        """CG coefficients (alpha, beta) of `steps` block-Jacobi PCG iterations on the probe vector."""
        a, b = np.zeros(steps), np.zeros(steps)
        j = lib().or_bj_lanczos(self._h, int(steps), a, b)
        if j < 0:
            raise RuntimeError("block-Jacobi Lanczos failed: singular block or K not SPD")
        return a[:j], b[:j]

    def cheb_bounds(self, steps, safety, ratio):
        """Interval of the Chebyshev preconditioner: hi = safety * (largest Ritz value of the
        Lanczos matrix of M^-1 K_t after `steps` iterations), lo = hi / ratio."""
        hi = safety * ritz_values(*self.bj_lanczos(steps))[-1]
        return hi / ratio, hi

    def prevost(self, b1, b2, tol_outer=1e-10, tol_inner=1e-12, maxit_outer=500, maxit_inner=200000):
        x1, x2, st = np.zeros(3 * self.N), np.zeros(self.N), np.zeros(5)
        s = lib().or_prevost(self._h, _c(b1, np.float64), _c(b2, np.float64), x1, x2, tol_outer, tol_inner,
                             maxit_outer, maxit_inner, st)
        return x1, x2, s, st

    def residual(self, U, P, Un, Pn, fcoh, Fu=None, fp=None):
        Fu = np.zeros(3 * self.N) if Fu is None else Fu
        fp = self.inst.source if fp is None else fp
        Rm, Rf = np.zeros(3 * self.N), np.zeros(self.N)
        lib().or_residual(self._h, *[_c(a, np.float64) for a in (U, P, Un, Pn, fcoh, Fu, fp)], Rm, Rf)
        return Rm, Rf

    def step(self, U, P, die, Fu=None, fp=None, tol_newton=1e-10, max_newton=30, tol_outer=1e-10,
             tol_inner=1e-12, maxit_outer=500, maxit_inner=200000, t0=None, line_search=True):
        """One implicit step; U, P, die are updated in place. Returns (trac, flag, info, status);
        info = (Newton iterations, outer, K and A22 inner iterations, scaled residuals m and f,
        status, step-length cuts of the line search)."""
        Fu = np.zeros(3 * self.N) if Fu is None else _c(Fu, np.float64)
        fp = self.inst.source if fp is None else _c(fp, np.float64)
        t0 = self.inst.t0 if t0 is None else t0
        nq = max(self.nq, 1)
        trac, flag, info = np.zeros(nq * 3), np.zeros(nq, np.uint8), np.zeros(8)
        dieb = np.zeros(nq * 2)
        dieb[: self.nq * 2] = die.reshape(-1)
        t0b = np.zeros(nq * 3)
        t0b[: self.nq * 3] = np.asarray(t0).reshape(-1)
        s = lib().or_step(self._h, U, P, dieb, trac, flag, t0b, Fu, fp, tol_newton, max_newton, tol_outer,
                          tol_inner, maxit_outer, maxit_inner, int(bool(line_search)), info)
        die.reshape(-1)[:] = dieb[: self.nq * 2]
        return trac.reshape(-1, 3)[: self.nq], flag[: self.nq], info, s


def _adjoint_methods():
    def apply_NT(self, x):
        """N^T x: transpose of the slip-tangent part the symmetric Newton tangent omits (last cohesive call)."""
        y = np.zeros(3 * self.N)
        lib().or_apply_NT(self._h, _c(x, np.float64), y)
        return y

    def apply_N(self, x):
        """N x: the slip-tangent part the symmetric Newton tangent omits (last cohesive call)."""
        y = np.zeros(3 * self.N)
        lib().or_apply_N(self._h, _c(x, np.float64), y)
        return y

    def bicgstab_exact(self, b, tol=1e-10, maxit=100000):
        """(K_t + N) x = b by BiCGStab with right block-Jacobi preconditioning: (x, status, iters, relres)."""
        x = np.zeros(3 * self.N)
        it, rr = C.c_int64(), C.c_double()
        st = lib().or_bicgstab_exact(self._h, _c(b, np.float64), x, tol, maxit, C.byref(it), C.byref(rr))
        return x, st, it.value, rr.value

    def adjoint(self, g_u, g_p, tol_defect=1e-12, max_defect=50, tol_outer=1e-12, tol_inner=1e-13,
                maxit_outer=1000, maxit_inner=500000):
        """(lam_u, lam_p, status, stats) of the transposed Newton system at the state of the last cohesive call."""
        lu, lp, st = np.zeros(3 * self.N), np.zeros(self.N), np.zeros(6)
        s = lib().or_adjoint(self._h, _c(g_u, np.float64), _c(g_p, np.float64), lu, lp, tol_defect, max_defect,
                             tol_outer, tol_inner, maxit_outer, maxit_inner, st)
        return lu, lp, s, st

    def sensitivity(self, U, P, lam_u, lam_p):
        """(dJ/dE, dJ/dlnk) per tetrahedron."""
        ne = self.inst.mesh.tets.shape[0]
        dE, dk = np.zeros(ne), np.zeros(ne)
        lib().or_sensitivity(self._h, *[_c(a, np.float64) for a in (U, P, lam_u, lam_p)], dE, dk)
        return dE, dk

    def slip_adjoint(self, U, die_old, a_new, lam_u=None, t0=None):
        """(gU, a_old) of the return map's slip-state adjoint (see or_slip_adjoint)."""
        t0 = self.inst.t0 if t0 is None else t0
        gU, a_old = np.zeros(3 * self.N), np.zeros(2 * max(self.nq, 1))
        lam = None if lam_u is None else _c(lam_u, np.float64)
        lib().or_slip_adjoint(self._h, _c(U, np.float64), _c(np.asarray(die_old).reshape(-1), np.float64),
                              _c(np.asarray(t0).reshape(-1), np.float64), _c(np.asarray(a_new).reshape(-1), np.float64),
                              None if lam is None else lam.ctypes.data, gU.ctypes.data, a_old.ctypes.data)
        return gU, a_old[: 2 * self.nq].reshape(-1, 2)

    def trajectory(self, steps, **step_kw):
        """Forward time loop of `steps` implicit steps from rest; returns the checkpoints
        [(U_n, P_n, die_{n-1}, die_n)] (the slip state carried from step to step)."""
        U, Pp, die = np.zeros(3 * self.N), np.zeros(self.N), np.zeros((self.nq, 2))
        ck = []
        for _ in range(steps):
            die_prev = die.copy()
            trac, flag, info, st = self.step(U, Pp, die, **step_kw)
            if st != 0:
                raise RuntimeError(f"oracle step failed with status {st}")
            ck.append((U.copy(), Pp.copy(), die_prev, die.copy()))
        return ck

    def trajectory_gradient(self, ck, grad_y, slip_state=True, **adj_kw):
        """dJ/dE, dJ/dln k of J = sum_n j_n(U_n, P_n) over the checkpointed loop, by the
        reverse sweep: for n = T..1, J_n^T lam_n = dj_n/dy_n - (dR_{n+1}/dy_n)^T lam_{n+1}
        + (dPhi_n/dU_n)^T a_n, with dR_{n+1,f}/dU_n = -A_up, dR_{n+1,f}/dP_n = -S (storage),
        then a_{n-1} = (dPhi_n/ddie_{n-1})^T a_n - (dR_n/ddie_{n-1})^T lam_n; the gradient
        sums -lam_n^T dR_n/dtheta.  grad_y(n, U, P) -> (dj/dU, dj/dP), n counted from 0.
        slip_state=False drops the slip-state terms (a_n = 0), for comparison only.
        The lagged slip term contracts slowly once slip spreads (about 0.87 per defect
        iteration at 18 of 96 points slipping), hence the larger default iteration cap."""
        adj_kw = {"max_defect": 1000, **adj_kw}
        dt = self.inst.params.dt
        a = np.zeros((self.nq, 2))
        lp_next = None
        dE_t, dk_t = 0.0, 0.0
        for n in range(len(ck) - 1, -1, -1):
            U, Pp, die_prev, _ = ck[n]
            gu, gp = (np.array(v, dtype=np.float64) for v in grad_y(n, U, Pp))
            if lp_next is not None:
                gu = gu + self.apply_Apu(lp_next)
                gp = gp + self.spmv(A22, lp_next) - dt * self.spmv(C_FLOW, lp_next)
            if slip_state:
                gu = gu + self.slip_adjoint(U, die_prev, a)[0]
            self.cohesive(U, die_prev)
            lu, lp, st, stats = self.adjoint(gu, gp, **adj_kw)
            if st != 0:
                raise RuntimeError(f"oracle adjoint failed with status {st}")
            dE, dk = self.sensitivity(U, Pp, lu, lp)
            dE_t, dk_t = dE_t + dE, dk_t + dk
            if slip_state:
                a = self.slip_adjoint(U, die_prev, a, lu)[1]
            lp_next = lp
        return dE_t, dk_t

    def pcg_amg(self, b, hi0, coarse_nodes=64, tol=1e-10, maxit=100000):
        """K_t x = b by PCG with the smoothed-aggregation V-cycle: (x, status, iters, relres, levels, nodes per level)."""
        x = np.zeros(3 * self.N)
        it, rr = C.c_int64(), C.c_double()
        st = np.zeros(7)
        s = lib().or_pcg_amg(self._h, _c(b, np.float64), x, tol, maxit, float(hi0), int(coarse_nodes), C.byref(it),
                             C.byref(rr), st)
        return x, s, it.value, rr.value, int(st[0]), st[1:1 + int(st[0])].astype(int)

    def amg_apply(self, r, hi0, coarse_nodes=64):
        """One V-cycle z = B r of the smoothed-aggregation preconditioner for the current K_t."""
        z = np.zeros(3 * self.N)
        s = lib().or_amg_apply(self._h, _c(r, np.float64), z, float(hi0), int(coarse_nodes))
        if s != 0:
            raise RuntimeError(f"AMG set-up failed ({s})")
        return z

    def amg_export(self, hi0, level, which, coarse_nodes=64):
        """Level `level` of the hierarchy: which 0 -> A_l, 1 -> P_l (scipy CSR), 2 -> aggregate of each node."""
        import scipy.sparse as sp
        dims = np.zeros(3, np.int64)
        if lib().or_amg_export(self._h, float(hi0), int(coarse_nodes), level, which, dims, None, None, None) == -1:
            raise IndexError(level)
        if which == 2:
            agg = np.zeros(dims[0], np.int32)
            lib().or_amg_export(self._h, float(hi0), int(coarse_nodes), level, which, dims, None, agg.ctypes.data, None)
            return agg
        rp, col, val = np.zeros(dims[0] + 1, np.int64), np.zeros(dims[2], np.int32), np.zeros(dims[2])
        lib().or_amg_export(self._h, float(hi0), int(coarse_nodes), level, which, dims, rp.ctypes.data,
                            col.ctypes.data, val.ctypes.data)
        return sp.csr_matrix((val, col, rp), shape=(int(dims[0]), int(dims[1])))

    Problem.pcg_amg = pcg_amg
    Problem.amg_apply = amg_apply
    Problem.amg_export = amg_export
    Problem.apply_NT = apply_NT
    Problem.apply_N = apply_N
    Problem.bicgstab_exact = bicgstab_exact
    Problem.adjoint = adjoint
    Problem.sensitivity = sensitivity
    Problem.slip_adjoint = slip_adjoint
    Problem.trajectory = trajectory
    Problem.trajectory_gradient = trajectory_gradient


_adjoint_methods()


def lanczos_matrix(alpha, beta):
    """Tridiagonal Lanczos matrix from CG coefficients (Saad, Sec. 6.7.3):
    T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j."""
    m = len(alpha)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(beta[j]) / alpha[j]
    return T


def ritz_values(alpha, beta):
    """Eigenvalues (ascending) of the Lanczos matrix of the CG coefficients."""
    return np.linalg.eigvalsh(lanczos_matrix(alpha, beta))


def num_threads() -> int:
    return lib().or_num_threads()
