"""Python binding of the lmfr C ABI (include/lmfr.h): argument marshalling only.

Every step of the residual, its derivatives, the preconditioner and the BDF2 step
runs in the HIP kernels of liblmfr.so; PyTorch provides device memory and streams.
Loading fails loudly when the library is missing or no HIP device is present.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmfr.so")
_lib = None

FR_OK, FR_EINVAL, FR_EHIP, FR_ENOMEM, FR_ENONFINITE, FR_ENOCONV, FR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FR_FP64, FR_FP32, FR_BF16 = 0, 1, 2
# boundary codes of the neighbour table (negative entries)
FR_BC_FARFIELD, FR_BC_SLIP_WALL, FR_BC_NOSLIP_WALL = -1, -2, -3
PREC = {"fp64": FR_FP64, "fp32": FR_FP32, "bf16": FR_BF16}

# every symbol declared in include/lmfr.h
EXPORTS = ["fr_create", "fr_set_geometry", "fr_residual", "fr_jvp", "fr_vjp", "fr_bdf_operator",
           "fr_block_jacobi_factor", "fr_block_jacobi_apply", "fr_get_blocks", "fr_bdf2_step",
           "fr_affine_elements", "fr_steady_solve", "fr_batch_steady_solve", "fr_set_farfield",
           "fr_set_option", "fr_autotune", "fr_batch_create", "fr_batch_destroy", "fr_batch_layout",
           "fr_batch_residual", "fr_batch_jvp", "fr_batch_bdf2_step", "fr_batch_set_option",
           "fr_batch_autotune", "fr_last_error", "fr_destroy", "fr_get_inverse", "fr_reserve",
           "fr_batch_reserve", "fr_vjp_noalloc"]


class FRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lmfr status {status}: {msg}")
        self.status = status


class fr_params(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("geom_order", ctypes.c_int32), ("n_elem", ctypes.c_int32),
                ("viscous", ctypes.c_int32), ("moving", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("mach_ref", ctypes.c_double), ("reynolds", ctypes.c_double),
                ("prandtl", ctypes.c_double), ("mu", ctypes.c_double), ("kappa", ctypes.c_double),
                ("mach_inf", ctypes.c_double)]


class fr_step_opts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("inv_dtau", ctypes.c_double), ("tol_pseudo", ctypes.c_double),
                ("tol_res", ctypes.c_double), ("tol_abs", ctypes.c_double), ("krylov", ctypes.c_int32),
                ("max_lin_it", ctypes.c_int32), ("max_newton", ctypes.c_int32), ("jac_lag", ctypes.c_int32),
                ("prec", ctypes.c_int32)]


class fr_step_stats(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int32), ("gmres_its", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("res0", ctypes.c_double), ("res_final", ctypes.c_double)]


class fr_steady_opts(ctypes.Structure):
    _fields_ = [("dtau0", ctypes.c_double), ("dtau_min", ctypes.c_double), ("dtau_max", ctypes.c_double),
                ("r_ser", ctypes.c_double), ("tol_pseudo", ctypes.c_double), ("tol_res", ctypes.c_double),
                ("tol_abs", ctypes.c_double), ("krylov", ctypes.c_int32), ("max_lin_it", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("jac_lag", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("reject_growth", ctypes.c_double)]


class fr_steady_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("gmres_its", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("res0", ctypes.c_double), ("res_final", ctypes.c_double), ("dtau_final", ctypes.c_double),
                ("rejected", ctypes.c_int32)]


def load_library(path: str = LIB_PATH):
    """Load liblmfr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"lmfr HIP library not built: {path} (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, dp = ctypes.c_void_p, ctypes.c_void_p
    L.fr_create.argtypes = [ctypes.POINTER(fr_params), vp, vp, vp, ctypes.POINTER(ctypes.c_void_p)]
    L.fr_set_geometry.argtypes = [vp, dp, dp, vp]
    L.fr_residual.argtypes = [vp, dp, dp, vp]
    L.fr_jvp.argtypes = [vp, dp, dp, dp, dp, vp]
    L.fr_vjp.argtypes = [vp, dp, dp, dp, vp]
    L.fr_vjp_noalloc.argtypes = [vp, dp, dp, dp, vp]
    L.fr_bdf_operator.argtypes = [vp, dp, dp, ctypes.c_double, ctypes.c_double, dp, vp]
    L.fr_block_jacobi_factor.argtypes = [vp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp]
    L.fr_block_jacobi_apply.argtypes = [vp, dp, dp, vp]
    L.fr_get_blocks.argtypes = [vp, dp, vp]
    L.fr_get_inverse.argtypes = [vp, dp, vp]
    L.fr_reserve.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.fr_batch_reserve.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.fr_affine_elements.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    L.fr_set_farfield.argtypes = [vp, dp]
    L.fr_steady_solve.argtypes = [vp, dp, ctypes.POINTER(fr_steady_opts), ctypes.POINTER(fr_steady_stats), vp]
    L.fr_batch_steady_solve.argtypes = [vp, vp, vp, vp, vp]
    L.fr_bdf2_step.argtypes = [vp, dp, dp, ctypes.POINTER(fr_step_opts), ctypes.POINTER(fr_step_stats), vp]
    L.fr_set_option.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64]
    L.fr_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    L.fr_batch_create.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
    L.fr_batch_destroy.argtypes = [vp]
    L.fr_batch_layout.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), vp]
    L.fr_batch_residual.argtypes = [vp, dp, dp, vp]
    L.fr_batch_jvp.argtypes = [vp, dp, dp, dp, vp]
    L.fr_batch_bdf2_step.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fr_batch_set_option.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64]
    L.fr_batch_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    L.fr_last_error.restype = ctypes.c_char_p
    L.fr_destroy.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("fr_last_error", "fr_destroy", "fr_batch_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != FR_OK:
        raise FRError(st, load_library().fr_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A discretisation context: mesh connectivity, geometry and physical parameters."""

    def __init__(self, prm, nbr, nbr_face, flip=None, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("lmfr needs a HIP device")
        L = load_library()
        self.device = torch.device(device)
        p = fr_params(int(prm.order), int(prm.geom_order), int(prm.n_elem), int(bool(prm.viscous)),
                      int(bool(prm.moving)), float(prm.gamma), float(prm.mach_ref), float(prm.reynolds),
                      float(prm.prandtl), float(prm.mu), float(prm.kappa), float(prm.mach_inf))
        self._nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        self._nbf = np.ascontiguousarray(nbr_face, dtype=np.int32)
        self._flip = None if flip is None else np.ascontiguousarray(flip, dtype=np.int8)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.fr_create(ctypes.byref(p), self._nbr.ctypes.data_as(ctypes.c_void_p),
                               self._nbf.ctypes.data_as(ctypes.c_void_p),
                               None if self._flip is None else self._flip.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(h)))
        self.h = h
        self.prm = prm
        self.E = int(prm.n_elem)
        self.Np = (int(prm.order) + 1) ** 2
        self.shape = (4, self.E, self.Np)

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                load_library().fr_destroy(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    def _dev(self, x):
        if x is None:
            return None
        t = torch.as_tensor(x, dtype=torch.float64, device=self.device)
        return t.contiguous()

    def _state(self, x):
        t = self._dev(x)
        if tuple(t.shape) != self.shape and t.numel() != 4 * self.E * self.Np:
            raise ValueError(f"state of shape {tuple(t.shape)}, expected {self.shape}")
        return t.view(self.shape)

    def set_geometry(self, xg, vg=None):
        self._xg = self._dev(xg)
        self._vg = self._dev(vg)
        _check(load_library().fr_set_geometry(self.h, _ptr(self._xg), _ptr(self._vg), _stream()))

    def set_option(self, name: str, value: int):
        _check(load_library().fr_set_option(self.h, name.encode(), int(value)))

    def residual(self, q, out=None):
        q = self._state(q)
        R = torch.empty_like(q) if out is None else out
        _check(load_library().fr_residual(self.h, _ptr(q), _ptr(R), _stream()))
        return R

    def jvp(self, q, v, want_residual=False, out=None):
        q, v = self._state(q), self._state(v)
        Jv = torch.empty_like(q) if out is None else out
        R = torch.empty_like(q) if want_residual else None
        _check(load_library().fr_jvp(self.h, _ptr(q), _ptr(v), _ptr(Jv), _ptr(R), _stream()))
        return (Jv, R) if want_residual else Jv

    def vjp(self, q, w, out=None):
        q, w = self._state(q), self._state(w)
        out = torch.empty_like(q) if out is None else out
        _check(load_library().fr_vjp(self.h, _ptr(q), _ptr(w), _ptr(out), _stream()))
        return out

    def bdf_operator(self, q, v, c_time, inv_dtau):
        q, v = self._state(q), self._state(v)
        out = torch.empty_like(q)
        _check(load_library().fr_bdf_operator(self.h, _ptr(q), _ptr(v), float(c_time), float(inv_dtau),
                                              _ptr(out), _stream()))
        return out

    def block_jacobi_factor(self, q, c_time, inv_dtau, prec="fp64"):
        q = self._state(q)
        _check(load_library().fr_block_jacobi_factor(self.h, _ptr(q), float(c_time), float(inv_dtau),
                                                     PREC[prec] if isinstance(prec, str) else int(prec),
                                                     _stream()))

    def block_jacobi_apply(self, r):
        r = self._state(r)
        z = torch.empty_like(r)
        _check(load_library().fr_block_jacobi_apply(self.h, _ptr(r), _ptr(z), _stream()))
        return z

    def set_farfield(self, qinf):
        """Free-stream primitive state (p, u, v, T) beyond the far-field boundary faces."""
        a = np.ascontiguousarray(qinf, dtype=np.float64).reshape(4)
        _check(load_library().fr_set_farfield(self.h, a.ctypes.data_as(ctypes.c_void_p)))

    def affine_elements(self):
        """Elements the last set_geometry found affine (constant metrics)."""
        n = ctypes.c_int32()
        _check(load_library().fr_affine_elements(self.h, ctypes.byref(n), _stream()))
        return n.value

    def get_blocks(self):
        nb = 4 * self.Np
        out = torch.empty((self.E, nb, nb), dtype=torch.float64, device=self.device)
        _check(load_library().fr_get_blocks(self.h, _ptr(out), _stream()))
        return out

    def get_inverse(self):
        """The stored inverse blocks of the last factor, widened to FP64, [E][4Np][4Np] row-major."""
        nb = 4 * self.Np
        out = torch.empty((self.E, nb, nb), dtype=torch.float64, device=self.device)
        _check(load_library().fr_get_inverse(self.h, _ptr(out), _stream()))
        return out

    def reserve(self, krylov_max, prec="fp64"):
        """Allocate every workspace of the factor, apply and step paths now (fr_reserve)."""
        _check(load_library().fr_reserve(self.h, int(krylov_max), PREC[prec] if isinstance(prec, str) else int(prec)))

    def autotune(self, cache_path=None):
        _check(load_library().fr_autotune(self.h, None if cache_path is None else str(cache_path).encode(),
                                          _stream()))

    def bdf2_step(self, q, q_nm1, dt, tol_pseudo=1e-8, tol_res=1e-6, krylov=30, max_lin_it=100,
                  max_newton=100, jac_lag=2, inv_dtau=1e-20, tol_abs=0.0, prec="fp64", check=True):
        """One BDF2 step in place on q (a float64 device tensor); returns the stats dict."""
        q = self._state(q)
        qn1 = None if q_nm1 is None else self._state(q_nm1)
        o = step_opts(dt, tol_pseudo, tol_res, krylov, max_lin_it, max_newton, jac_lag, inv_dtau, tol_abs, prec)
        st = fr_step_stats()
        rc = load_library().fr_bdf2_step(self.h, _ptr(q), _ptr(qn1), ctypes.byref(o), ctypes.byref(st), _stream())
        if check and rc not in (FR_OK, FR_ENOCONV):
            _check(rc)
        return dict(rc=rc, newton_its=st.newton_its, gmres_its=st.gmres_its, converged=st.converged,
                    res0=st.res0, res_final=st.res_final)

    def steady_solve(self, q, check=True, **kw):
        """Steady pseudo-transient solve in place on q; keywords as steady_opts.  Returns stats."""
        q = self._state(q)
        o = steady_opts(**kw)
        st = fr_steady_stats()
        rc = load_library().fr_steady_solve(self.h, _ptr(q), ctypes.byref(o), ctypes.byref(st), _stream())
        if check and rc not in (FR_OK, FR_ENOCONV):
            _check(rc)
        return dict(rc=rc, **_steady_dict(st))


def steady_opts(dtau0=0.01, dtau_min=0.01, dtau_max=1e20, r_ser=2.0, tol_pseudo=1e-8, tol_res=1e-6, tol_abs=0.0,
                krylov=30, max_lin_it=200, max_steps=100, jac_lag=1, prec="fp64", reject_growth=0.0):
    """Options of a steady pseudo-transient solve (paper defaults for the SER controls; step
    rejection, which is not part of the paper's method, off unless reject_growth > 0)."""
    return fr_steady_opts(float(dtau0), float(dtau_min), float(dtau_max), float(r_ser), float(tol_pseudo),
                          float(tol_res), float(tol_abs), int(krylov), int(max_lin_it), int(max_steps), int(jac_lag),
                          PREC[prec] if isinstance(prec, str) else int(prec), float(reject_growth))


def _steady_dict(s):
    return dict(steps=s.steps, gmres_its=s.gmres_its, converged=s.converged, res0=s.res0, res_final=s.res_final,
                dtau_final=s.dtau_final, rejected=s.rejected)


def step_opts(dt, tol_pseudo=1e-8, tol_res=1e-6, krylov=30, max_lin_it=100, max_newton=100, jac_lag=2,
              inv_dtau=1e-20, tol_abs=0.0, prec="fp64"):
    return fr_step_opts(float(dt), float(inv_dtau), float(tol_pseudo), float(tol_res), float(tol_abs),
                        int(krylov), int(max_lin_it), int(max_newton), int(jac_lag),
                        PREC[prec] if isinstance(prec, str) else int(prec))


class Batch:
    """Many contexts advanced together (fr_batch_*): one launch per kind of case."""

    def __init__(self, contexts):
        L = load_library()
        self.contexts = list(contexts)
        arr = (ctypes.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = ctypes.c_void_p()
        _check(L.fr_batch_create(arr, len(self.contexts), ctypes.byref(h)))
        self.h = h
        n_total = ctypes.c_int64()
        offs = (ctypes.c_int64 * len(self.contexts))()
        _check(L.fr_batch_layout(self.h, ctypes.byref(n_total), offs))
        self.n_total = int(n_total.value)
        self.offsets = [int(x) for x in offs]
        self.device = self.contexts[0].device

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                load_library().fr_batch_destroy(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    def pack(self, states):
        """Concatenate per-case states into the batch layout (zero padding)."""
        out = torch.zeros(self.n_total, dtype=torch.float64, device=self.device)
        for c, (ctx, x) in enumerate(zip(self.contexts, states)):
            n = 4 * ctx.E * ctx.Np
            out[self.offsets[c]:self.offsets[c] + n] = ctx._state(x).reshape(-1)
        return out

    def unpack(self, flat):
        return [flat[o:o + 4 * c.E * c.Np].view(c.shape) for c, o in zip(self.contexts, self.offsets)]

    def residual(self, q_flat, out=None):
        R = torch.zeros_like(q_flat) if out is None else out
        _check(load_library().fr_batch_residual(self.h, _ptr(q_flat), _ptr(R), _stream()))
        return R

    def jvp(self, q_flat, v_flat):
        Jv = torch.zeros_like(q_flat)
        _check(load_library().fr_batch_jvp(self.h, _ptr(q_flat), _ptr(v_flat), _ptr(Jv), _stream()))
        return Jv

    def set_option(self, name: str, value: int):
        _check(load_library().fr_batch_set_option(self.h, name.encode(), int(value)))

    def reserve(self, krylov_max, prec="fp64"):
        _check(load_library().fr_batch_reserve(self.h, int(krylov_max),
                                               PREC[prec] if isinstance(prec, str) else int(prec)))

    def autotune(self, cache_path=None):
        _check(load_library().fr_batch_autotune(self.h, None if cache_path is None else str(cache_path).encode(),
                                                _stream()))

    def bdf2_step(self, qs, q_nm1s, opts, check=True):
        """One step of every case in place on the tensors qs; opts: one fr_step_opts per case
        (or one shared).  Returns (status, [stats dicts])."""
        n = len(self.contexts)
        if isinstance(opts, fr_step_opts):
            opts = [opts] * n
        qs = [c._state(q) for c, q in zip(self.contexts, qs)]
        qarr = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
        if q_nm1s is None:
            parr = None
        else:
            pm = [None if x is None else c._state(x) for c, x in zip(self.contexts, q_nm1s)]
            self._keep = pm
            parr = (ctypes.c_void_p * n)(*[None if x is None else x.data_ptr() for x in pm])
        oarr = (fr_step_opts * n)(*opts)
        sarr = (fr_step_stats * n)()
        rc = load_library().fr_batch_bdf2_step(self.h, qarr, parr, oarr, sarr, _stream())
        if check and rc not in (FR_OK, FR_ENOCONV):
            _check(rc)
        return rc, [dict(newton_its=s.newton_its, gmres_its=s.gmres_its, converged=s.converged, res0=s.res0,
                         res_final=s.res_final) for s in sarr]

    def steady_solve(self, qs, opts, check=True):
        """Steady solve of every case in place on the tensors qs; opts: one fr_steady_opts per
        case (or one shared).  Returns (status, [stats dicts])."""
        n = len(self.contexts)
        if isinstance(opts, fr_steady_opts):
            opts = [opts] * n
        qs = [c._state(q) for c, q in zip(self.contexts, qs)]
        qarr = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
        oarr = (fr_steady_opts * n)(*opts)
        sarr = (fr_steady_stats * n)()
        rc = load_library().fr_batch_steady_solve(self.h, qarr, oarr, sarr, _stream())
        if check and rc not in (FR_OK, FR_ENOCONV):
            _check(rc)
        return rc, [_steady_dict(s) for s in sarr]


def _plain(t):
    """The tensor under torch.func's wrappers (torch.func.jvp hands the jvp rule wrapped
    tensors, which have no storage for the kernels to read)."""
    from torch._C._functorch import get_unwrapped, is_functorch_wrapped_tensor
    while is_functorch_wrapped_tensor(t):
        t = get_unwrapped(t)
    return t


class FRResidual(torch.autograd.Function):
    """R(q) with exact derivatives: forward = fr_residual, backward = fr_vjp, jvp = fr_jvp."""

    @staticmethod
    def forward(q, ctx_fr):
        return ctx_fr.residual(q)

    @staticmethod
    def setup_context(ctx, inputs, output):
        q, ctx_fr = inputs
        ctx.save_for_backward(q)
        ctx.save_for_forward(q)
        ctx.fr = ctx_fr

    @staticmethod
    def backward(ctx, w):
        (q,) = ctx.saved_tensors
        return ctx.fr.vjp(q, w.contiguous()), None

    @staticmethod
    def jvp(ctx, v, _):
        (q,) = ctx.saved_tensors
        with torch._C._DisableFuncTorch():   # the binding's own tensor ops stay unwrapped
            return ctx.fr.jvp(_plain(q), _plain(v).contiguous())


def residual(q, ctx_fr):
    return FRResidual.apply(q, ctx_fr)


# ----------------------------------------------------------------------------- checkpoint / resume
CHECKPOINT_FORMAT = "lmfr-bdf2-state-1"


def save_checkpoint(path, q, q_nm1, t, dt, step=0):
    """Write the state a BDF2 march needs to continue (paper Sec. 3.2: the step from t to t + dt
    reads q^n and q^{n-1}) to a safetensors file: the states as float64 host copies, and t, dt and
    the step count as metadata (exact decimal round trip).

    q, q_nm1: one context's state tensors, or lists of them for a batch; q_nm1 may be None (the
    next step is then a BDF1 start).  A step also depends on the geometry at t + dt and on the
    step options, which the caller sets again when it resumes; the preconditioner is refreshed at
    the first Newton iteration of every step, so no solver state has to be saved."""
    from safetensors.torch import save_file
    many = isinstance(q, (list, tuple))
    qs = list(q) if many else [q]
    if q_nm1 is None:
        ms = [None] * len(qs)
    else:
        ms = list(q_nm1) if many else [q_nm1]
    if len(ms) != len(qs):
        raise ValueError("q and q_nm1 hold different numbers of states")
    tensors = {}
    for i, (a, b) in enumerate(zip(qs, ms)):
        tensors[f"q.{i}"] = a.detach().to("cpu", torch.float64).contiguous()
        if b is not None:
            tensors[f"q_nm1.{i}"] = b.detach().to("cpu", torch.float64).contiguous()
    meta = {"format": CHECKPOINT_FORMAT, "t": repr(float(t)), "dt": repr(float(dt)), "step": str(int(step)),
            "count": str(len(qs)), "batch": "1" if many else "0", "has_nm1": "0" if q_nm1 is None else "1"}
    save_file(tensors, str(path), metadata=meta)


def load_checkpoint(path, device="cuda"):
    """Read what save_checkpoint wrote: a dict with q, q_nm1 (tensors on `device`, lists for a
    batch, q_nm1 None for a BDF1 start), t, dt and step."""
    from safetensors import safe_open
    with safe_open(str(path), framework="pt", device="cpu") as f:
        meta = f.metadata() or {}
        if meta.get("format") != CHECKPOINT_FORMAT:
            raise ValueError(f"{path}: not an lmfr BDF2 checkpoint")
        n = int(meta["count"])
        qs = [f.get_tensor(f"q.{i}").to(device) for i in range(n)]
        ms = [f.get_tensor(f"q_nm1.{i}").to(device) for i in range(n)] if meta["has_nm1"] == "1" else None
    batch = meta["batch"] == "1"
    return {"q": qs if batch else qs[0], "q_nm1": (ms if batch else ms[0]) if ms is not None else None,
            "t": float(meta["t"]), "dt": float(meta["dt"]), "step": int(meta["step"])}
