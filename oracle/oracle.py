"""ORACLE -- test infrastructure only (ctypes wrapper of oracle/fr_oracle.cpp).

A plain serial FP64 CPU implementation of the implicit preconditioned FR/CPR
method, written from the paper. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module. It shares no code with the
GPU library and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fr_oracle.cpp")
# a build of the same source with other flags (the CPU baseline's optimised OpenMP build)
# may be named by LMFR_ORACLE_LIB
_LIB = os.environ.get("LMFR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, serial, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
               "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_native(path: str) -> str:
    """The same source at -O3 -march=native with OpenMP element loops (no fast-math): the
    build the CPU baseline times, on the machine that runs it."""
    cmd = ["g++", "-O3", "-march=native", "-fopenmp", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
           "-o", path + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    return path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_destroy.argtypes = [ctypes.c_void_p]
        L.ora_set_threads.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_count_residual.restype = ctypes.c_int
        L.ora_openmp.restype = ctypes.c_int
        for name in ["ora_residual", "ora_jvp", "ora_dense_jacobian", "ora_vjp_dofs", "ora_blocks",
                     "ora_point", "ora_common_flux", "ora_phys_flux", "ora_bdf2_step", "ora_steady_solve", "ora_precond_apply",
                     "ora_geometry", "ora_scalar_residual", "ora_residual_cplx", "ora_cons_cplx"]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


def operators(p: int, pg: int | None = None):
    """1-D operators: GL nodes/weights, D[i,a] = l_a'(xi_i), face interpolation, Radau g', GLL nodes."""
    pg = p if pg is None else pg
    n = p + 1
    xi, w, lamL, lamR, gL, gR = (np.zeros(n) for _ in range(6))
    D = np.zeros((n, n))
    gll = np.zeros(pg + 1)
    lib().ora_operators(p, pg, _p(xi), _p(w), _p(D), _p(lamL), _p(lamR), _p(gL), _p(gR), _p(gll))
    return dict(xi=xi, w=w, D=D, lamL=lamL, lamR=lamR, gamL=gL, gamR=gR, gll=gll)


def lu_factor(A):
    A = np.array(A, dtype=np.float64, order="C")
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    rc = lib().ora_lu_factor(n, _p(A), _p(piv, _ip))
    return A, piv, rc


def lu_solve(LU, piv, b):
    b = np.array(b, dtype=np.float64)
    lib().ora_lu_solve(LU.shape[0], _p(LU), _p(piv, _ip), _p(b))
    return b


def gmres_dense(A, b, m=20, tol=1e-10, max_it=200, Pinv=None):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = len(b)
    x = np.zeros(n)
    its = ctypes.c_int(0)
    rel = ctypes.c_double(0)
    P = None if Pinv is None else np.ascontiguousarray(Pinv, dtype=np.float64)
    lib().ora_gmres_dense(n, _p(A), _p(P), _p(b), _p(x), m, ctypes.c_double(tol), max_it,
                          ctypes.byref(its), ctypes.byref(rel))
    return x, its.value, rel.value


class Oracle:
    """One discretisation context (mesh, geometry, physical parameters)."""

    def __init__(self, prm, mesh, xg=None, vg=None, t=0.0):
        self.prm, self.mesh = prm, mesh
        nbr, nbr_face, flip = mesh.connectivity()
        if xg is None:
            xg, vg = mesh.nodes(t)
        self.E, self.n, self.Np = mesh.E, prm.order + 1, (prm.order + 1) ** 2
        d = np.array([prm.gamma, prm.mach_ref, prm.reynolds, prm.prandtl, prm.mu, prm.kappa,
                      prm.mach_inf], dtype=np.float64)
        i = np.array([prm.order, prm.geom_order, mesh.E, int(prm.viscous), int(prm.moving)],
                     dtype=np.int32)
        self._keep = [np.ascontiguousarray(a) for a in (d, i, nbr, nbr_face, flip, xg)]
        vg_ = None if vg is None else np.ascontiguousarray(vg, dtype=np.float64)
        self._keep.append(vg_)
        k = self._keep
        self.h = ctypes.c_void_p(lib().ora_create(
            _p(k[0]), _p(k[1], _ip), _p(k[2], _ip), _p(k[3], _ip),
            k[4].ctypes.data_as(ctypes.POINTER(ctypes.c_byte)), _p(k[5]), _p(vg_)))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ora_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def N(self):
        return 4 * self.E * self.Np

    def _state(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.size == self.N, (q.shape, self.N)
        return q

    def set_farfield(self, qinf):
        """Free-stream primitive state (p, u, v, T) seen through the far-field boundary faces."""
        a = np.ascontiguousarray(qinf, dtype=np.float64).reshape(4)
        lib().ora_set_farfield(self.h, _p(a))

    def geometry(self):
        out = np.zeros((9, self.E, self.Np))
        fout = np.zeros((5, self.E, 4, self.n))
        lib().ora_geometry(self.h, _p(out), _p(fout))
        keys = ["x", "y", "jac", "xix", "xiy", "etx", "ety", "ug", "vg"]
        g = {k: out[i] for i, k in enumerate(keys)}
        for i, k in enumerate(["Sx", "Sy", "Jf", "ugf", "vgf"]):
            g[k] = fout[i]
        return g

    def residual(self, q):
        q = self._state(q)
        R = np.zeros_like(q)
        lib().ora_residual(self.h, _p(q), _p(R))
        return R

    def set_threads(self, n: int):
        """Element-loop threads of the residual (effective in an OpenMP build only)."""
        lib().ora_set_threads(self.h, int(n))

    def count_residual(self, q):
        """R on the op-counting scalar: (R, {add, mul, div, sqrt}) for one evaluation."""
        q = self._state(q)
        R = np.zeros_like(q)
        cnt = np.zeros(4, dtype=np.uint64)
        lib().ora_count_residual(self.h, _p(q), _p(R), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_ulonglong)))
        return R, dict(zip(["add", "mul", "div", "sqrt"], (int(x) for x in cnt)))

    def residual_complex(self, q):
        qr = np.ascontiguousarray(q.real, dtype=np.float64)
        qi = np.ascontiguousarray(q.imag, dtype=np.float64)
        Rr, Ri = np.zeros_like(qr), np.zeros_like(qr)
        lib().ora_residual_cplx(self.h, _p(qr), _p(qi), _p(Rr), _p(Ri))
        return Rr + 1j * Ri

    def scalar_residual(self, u, ax, ay, nu):
        u = np.ascontiguousarray(u, dtype=np.float64)
        R = np.zeros_like(u)
        lib().ora_scalar_residual(self.h, ctypes.c_double(ax), ctypes.c_double(ay),
                                  ctypes.c_double(nu), _p(u), _p(R))
        return R

    def jvp(self, q, v):
        q, v = self._state(q), self._state(v)
        out = np.zeros_like(q)
        lib().ora_jvp(self.h, _p(q), _p(v), _p(out))
        return out

    def dense_jacobian(self, q):
        q = self._state(q)
        J = np.zeros((self.N, self.N))
        lib().ora_dense_jacobian(self.h, _p(q), _p(J))
        return J

    def vjp_dofs(self, q, w, dofs):
        q, w = self._state(q), self._state(w)
        dofs = np.ascontiguousarray(dofs, dtype=np.int64)
        out = np.zeros(len(dofs))
        lib().ora_vjp_dofs(self.h, _p(q), _p(w), dofs.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                           ctypes.c_longlong(len(dofs)), _p(out))
        return out

    def blocks(self, q, c_time, inv_dtau, elements=None):
        q = self._state(q)
        nb = 4 * self.Np
        els = None if elements is None else np.ascontiguousarray(elements, dtype=np.int32)
        cnt = self.E if els is None else len(els)
        B = np.zeros((cnt, nb, nb))
        lib().ora_blocks(self.h, _p(q), ctypes.c_double(c_time), ctypes.c_double(inv_dtau),
                         _p(els, _ip), cnt, _p(B))
        return B

    def point(self, q, nx=1.0, ny=0.0, ug=0.0, vg=0.0):
        q = np.ascontiguousarray(q, dtype=np.float64)
        aux = np.array([nx, ny, ug, vg], dtype=np.float64)
        qc, fn = np.zeros(4), np.zeros(4)
        M, G = np.zeros(16), np.zeros(16)
        lam = ctypes.c_double(0)
        lib().ora_point(self.h, _p(q), _p(aux), _p(qc), _p(M), _p(G), _p(fn), ctypes.byref(lam))
        return dict(qc=qc, M=M.reshape(4, 4), Gamma=G.reshape(4, 4), fn=fn, lam=lam.value)

    def cons_complex(self, q):
        qr = np.ascontiguousarray(q.real, dtype=np.float64)
        qi = np.ascontiguousarray(q.imag, dtype=np.float64)
        orr, oi = np.zeros(4), np.zeros(4)
        lib().ora_cons_cplx(self.h, _p(qr), _p(qi), _p(orr), _p(oi))
        return orr + 1j * oi

    def common_flux(self, qL, qR, gxL, gyL, gxR, gyR, nx, ny, Smag=1.0, JfL=1.0, JfR=1.0, ug=0.0, vg=0.0):
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (qL, qR, gxL, gyL, gxR, gyR)]
        aux = np.array([nx, ny, Smag, JfL, JfR, ug, vg], dtype=np.float64)
        fn, qcom = np.zeros(4), np.zeros(4)
        lib().ora_common_flux(self.h, *[_p(x) for x in a], _p(aux), _p(fn), _p(qcom))
        return fn, qcom

    def phys_flux(self, q, gx, gy):
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (q, gx, gy)]
        f, g = np.zeros(4), np.zeros(4)
        lib().ora_phys_flux(self.h, *[_p(x) for x in a], _p(f), _p(g))
        return f, g

    def bdf2_step(self, q, q_nm1, dt, tol_pseudo=1e-8, tol_res=1e-6, krylov=30, max_lin_it=100,
                  max_newton=100, jac_lag=2, inv_dtau=1e-20, tol_abs=0.0, precond=0):
        q = np.array(self._state(q), copy=True)
        qn1 = None if q_nm1 is None else self._state(q_nm1)
        d = np.array([dt, inv_dtau, tol_pseudo, tol_res, tol_abs], dtype=np.float64)
        i = np.array([krylov, max_lin_it, max_newton, jac_lag, precond], dtype=np.int32)
        ist = np.zeros(3, dtype=np.int32)
        dst = np.zeros(2)
        rc = lib().ora_bdf2_step(self.h, _p(q), _p(qn1), _p(d), _p(i, _ip), _p(ist, _ip), _p(dst))
        stats = dict(rc=rc, newton_its=int(ist[0]), gmres_its=int(ist[1]), converged=int(ist[2]),
                     res0=float(dst[0]), res_final=float(dst[1]))
        return q, stats

    def steady_solve(self, q, dtau0=0.01, dtau_min=0.01, dtau_max=1e20, r_ser=2.0, tol_pseudo=1e-8,
                     tol_res=1e-6, tol_abs=0.0, krylov=30, max_lin_it=200, max_steps=100, jac_lag=1, precond=0,
                     reject_growth=0.0):
        """Steady pseudo-transient continuation with SER (Sec. 3.2): returns the final state and
        stats, with hist = [(Res_m, dtau_m)] of every pseudo-step taken."""
        q = np.array(self._state(q), copy=True)
        d = np.array([dtau0, dtau_min, dtau_max, r_ser, tol_pseudo, tol_res, tol_abs, reject_growth], dtype=np.float64)
        i = np.array([krylov, max_lin_it, max_steps, jac_lag, precond], dtype=np.int32)
        ist = np.zeros(4, dtype=np.int32)
        dst = np.zeros(3)
        hist = np.zeros(2 * (max_steps + 1))
        rc = lib().ora_steady_solve(self.h, _p(q), _p(d), _p(i, _ip), _p(ist, _ip), _p(dst), _p(hist))
        n = int(ist[0])
        stats = dict(rc=rc, steps=n, gmres_its=int(ist[1]), converged=int(ist[2]), rejected=int(ist[3]), res0=float(dst[0]),
                     res_final=float(dst[1]), dtau_final=float(dst[2]),
                     hist=[(float(hist[2 * k]), float(hist[2 * k + 1])) for k in range(n)])
        return q, stats

    def precond_apply(self, q, r, c_time, inv_dtau, precond=1):
        """z = P^-1 r for the Newton operator at q (precond 0: block Jacobi, 1: symmetric block
        Gauss-Seidel in colour order, 2: forward block Gauss-Seidel in colour order); returns
        (z, element colours)."""
        q = self._state(q)
        r = self._state(r)
        z = np.zeros_like(q)
        col = np.zeros(self.prm.n_elem, dtype=np.int32)
        rc = lib().ora_precond_apply(self.h, _p(q), ctypes.c_double(c_time), ctypes.c_double(inv_dtau), int(precond),
                                     _p(r), _p(z), _p(col, _ip))
        if rc != 0:
            raise RuntimeError(f"ora_precond_apply failed: {rc}")
        return z, col
