"""ctypes binding of liblindx (include/lind.h) on torch tensors.

Argument marshalling only: every step of every call runs in the HIP library.  Tensors must be
contiguous complex128 tensors on a CUDA(HIP) device; calls are enqueued on torch's current
stream.  If the library is not built or no gfx950 device is present, construction raises --
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblindx.so")

LIND_OK, LIND_EINVAL, LIND_ESINGULAR, LIND_ENOCONV, LIND_EDEVICE, LIND_ENOMEM = 0, -1, -2, -3, -4, -5
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
METHOD = {"phi_arnoldi": 0, "gmres": 1}
ROUTE = {"auto": 0, "eig": 1, "schur": 2}
SYMBOLS = ["lind_default_opts", "lind_create", "lind_destroy", "lind_apply", "lind_apply_adjoint", "lind_sinv",
           "lind_phi", "lind_steady_state", "lind_eigs", "lind_steady_grad", "lind_resolve", "lind_ie",
           "lind_factor_ptr", "lind_last_error", "lind_apply_noalloc", "lind_apply_noalloc_bytes"]


class LindOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("route", ctypes.c_int), ("kappa_max", ctypes.c_double),
                ("m", ctypes.c_int), ("p", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("refine_max", ctypes.c_int), ("eta", ctypes.c_double), ("time_limit_s", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("method", ctypes.c_int), ("gauge", ctypes.POINTER(ctypes.c_double))]


class LindInfo(ctypes.Structure):
    _fields_ = [("resid_trace", ctypes.c_double), ("resid_max", ctypes.c_double), ("err_est", ctypes.c_double),
                ("kappa_U", ctypes.c_double), ("t_factor_s", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("n_phi", ctypes.c_int), ("n_restarts", ctypes.c_int), ("n_refine", ctypes.c_int),
                ("n_inner", ctypes.c_int), ("route_used", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LindError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lindx error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblindx.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2608_30860_amd.build`")
    lib = ctypes.CDLL(path)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.lind_default_opts.argtypes = [ctypes.POINTER(LindOpts)]
    lib.lind_default_opts.restype = None
    lib.lind_create.argtypes = [ctypes.POINTER(vp), vp, vp, ci, ci, ctypes.POINTER(LindOpts)]
    lib.lind_create.restype = ci
    lib.lind_destroy.argtypes = [vp]
    lib.lind_destroy.restype = None
    for name in ["lind_apply", "lind_apply_adjoint", "lind_phi"]:
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp]
        f.restype = ci
    lib.lind_apply_noalloc.argtypes = [vp, vp, vp]
    lib.lind_apply_noalloc.restype = ci
    lib.lind_apply_noalloc_bytes.argtypes = [ci, ci]
    lib.lind_apply_noalloc_bytes.restype = ctypes.c_longlong
    lib.lind_sinv.argtypes = [vp, vp, vp, cd, cd]
    lib.lind_sinv.restype = ci
    lib.lind_steady_state.argtypes = [vp, cd, vp, vp, ctypes.POINTER(LindInfo)]
    lib.lind_steady_state.restype = ci
    lib.lind_eigs.argtypes = [vp, ci, cd, cd, cd, vp, vp, ctypes.POINTER(LindInfo)]
    lib.lind_eigs.restype = ci
    lib.lind_steady_grad.argtypes = [vp, vp, cd, ctypes.POINTER(cd), vp, vp, vp, ctypes.POINTER(LindInfo)]
    lib.lind_steady_grad.restype = ci
    lib.lind_resolve.argtypes = [vp, cd, cd, vp, vp, cd, ctypes.POINTER(LindInfo)]
    lib.lind_resolve.restype = ci
    lib.lind_ie.argtypes = [vp, cd, ci, vp, vp, cd, ctypes.POINTER(LindInfo)]
    lib.lind_ie.restype = ci
    lib.lind_factor_ptr.argtypes = [vp, ci]
    lib.lind_factor_ptr.restype = vp
    lib.lind_last_error.argtypes = [vp]
    lib.lind_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check_mat(t, n, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.shape[-2:] != (n, n) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with trailing shape ({n}, {n})")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SteadyResult:
    rho: torch.Tensor
    info: dict


class Lindblad:
    """A Lindbladian on one GPU: L(rho) = -i[H, rho] + sum_j (L_j rho L_j^+ - 1/2 {L_j^+ L_j, rho}).

    H: (n, n) complex128 CUDA tensor; Ls: (d, n, n) complex128 CUDA tensor or a list of (n, n).
    Options mirror lind_opts: prec ('fp64' | 'fp32' | 'bf16x3'), route ('auto' | 'eig' | 'schur'),
    kappa_max, m, p, max_restarts, refine_max, eta, time_limit_s, method ('phi_arnoldi' | 'gmres')
    and gauge (None or d complex shifts c_j of the no-jump / jump split).
    """

    def __init__(self, H, Ls, prec="fp64", route="auto", kappa_max=1e3, m=30, p=0, max_restarts=200,
                 refine_max=8, eta=1.0, time_limit_s=0.0, stream=None, method="phi_arnoldi", gauge=None):
        self.lib = load_library()
        if isinstance(Ls, (list, tuple)):
            Ls = torch.stack(list(Ls)) if len(Ls) else torch.zeros((0,) + tuple(H.shape), dtype=H.dtype, device=H.device)
        n = H.shape[0]
        _check_mat(H, n, "H")
        if Ls.numel():
            _check_mat(Ls, n, "Ls")
        Ls = Ls.contiguous()
        self.n, self.d = n, Ls.shape[0]
        self.device = H.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(H.device)
        o = LindOpts()
        self.lib.lind_default_opts(ctypes.byref(o))
        o.prec, o.route, o.kappa_max, o.m, o.p = PREC[prec], ROUTE[route], kappa_max, m, p
        o.max_restarts, o.refine_max, o.eta, o.time_limit_s = max_restarts, refine_max, eta, time_limit_s
        o.stream = ctypes.c_void_p(self.stream.cuda_stream)
        o.method = METHOD[method]
        if gauge is not None:
            cs = [complex(z) for z in gauge]
            if len(cs) != self.d:
                raise ValueError(f"gauge needs one shift per jump operator ({self.d})")
            self._gauge = (ctypes.c_double * (2 * len(cs)))(*[v for z in cs for v in (z.real, z.imag)])
            o.gauge = ctypes.cast(self._gauge, ctypes.POINTER(ctypes.c_double))
        self._opts = o
        h = ctypes.c_void_p()
        lptr = _ptr(Ls) if self.d else ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            rc = self.lib.lind_create(ctypes.byref(h), _ptr(H), lptr, n, self.d, ctypes.byref(o))
        if rc != LIND_OK:
            raise LindError(rc, self.lib.lind_last_error(None).decode())
        self.h = h
        self._keep = (H, Ls)

    # -------------------------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.lind_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc):
        raise LindError(rc, self.lib.lind_last_error(self.h).decode())

    def _new(self, *shape):
        return torch.empty(shape or (self.n, self.n), dtype=torch.complex128, device=self.device)

    def apply(self, rho):
        _check_mat(rho, self.n, "rho")
        out = self._new()
        rc = self.lib.lind_apply(self.h, _ptr(rho), _ptr(out))
        if rc:
            self._err(rc)
        return out

    def apply_noalloc(self, rho, out):
        """out = L(rho) through lind_apply_noalloc (intermediates in the library's fixed device
        array; the output buffer is the caller's)."""
        _check_mat(rho, self.n, "rho")
        _check_mat(out, self.n, "out")
        rc = self.lib.lind_apply_noalloc(self.h, _ptr(rho), _ptr(out))
        if rc:
            self._err(rc)
        return out

    def apply_adjoint(self, X):
        _check_mat(X, self.n, "X")
        out = self._new()
        rc = self.lib.lind_apply_adjoint(self.h, _ptr(X), _ptr(out))
        if rc:
            self._err(rc)
        return out

    def sinv(self, Y, mu=0.0):
        """X = (S - mu)^{-1} Y."""
        _check_mat(Y, self.n, "Y")
        out = self._new()
        mu = complex(mu)
        rc = self.lib.lind_sinv(self.h, _ptr(Y), _ptr(out), mu.real, mu.imag)
        if rc:
            self._err(rc)
        return out

    def phi(self, xi):
        _check_mat(xi, self.n, "xi")
        out = self._new()
        rc = self.lib.lind_phi(self.h, _ptr(xi), _ptr(out))
        if rc:
            self._err(rc)
        return out

    def steady_state(self, tol=1e-10, rho0=None, raise_on_noconv=True):
        out = self._new()
        info = LindInfo()
        r0 = ctypes.c_void_p(0)
        if rho0 is not None:
            _check_mat(rho0, self.n, "rho0")
            r0 = _ptr(rho0)
        rc = self.lib.lind_steady_state(self.h, tol, r0, _ptr(out), ctypes.byref(info))
        if rc and not (rc == LIND_ENOCONV and not raise_on_noconv):
            self._err(rc)
        d = info.as_dict()
        d["status"] = rc
        return SteadyResult(out, d)

    def eigs(self, k, mu=0.0, tol=1e-10, vectors=False, raise_on_noconv=True):
        ev = (ctypes.c_double * (2 * k))()
        vec = self._new(k, self.n, self.n) if vectors else None
        info = LindInfo()
        mu = complex(mu)
        rc = self.lib.lind_eigs(self.h, k, mu.real, mu.imag, tol, ctypes.cast(ev, ctypes.c_void_p),
                                _ptr(vec) if vec is not None else ctypes.c_void_p(0), ctypes.byref(info))
        if rc and not (rc == LIND_ENOCONV and not raise_on_noconv):
            self._err(rc)
        vals = np.array(ev[0::2]) + 1j * np.array(ev[1::2])
        d = info.as_dict()
        d["status"] = rc
        return vals, vec, d

    def steady_grad(self, O, tol=1e-12, want_rho=True):
        _check_mat(O, self.n, "O")
        gH = self._new()
        gL = self._new(max(self.d, 1), self.n, self.n)
        rho = self._new() if want_rho else None
        val = ctypes.c_double(0)
        info = LindInfo()
        rc = self.lib.lind_steady_grad(self.h, _ptr(O), tol, ctypes.byref(val), _ptr(gH), _ptr(gL),
                                       _ptr(rho) if rho is not None else ctypes.c_void_p(0), ctypes.byref(info))
        if rc:
            self._err(rc)
        return val.value, gH, gL[: self.d], rho, info.as_dict()

    def resolve(self, lam, B, tol=1e-12, raise_on_noconv=True):
        """X = (lam - L)^{-1} B, Re(lam) > 0 (lind_resolve).  Returns (X, info)."""
        _check_mat(B, self.n, "B")
        X = self._new()
        info = LindInfo()
        lam = complex(lam)
        rc = self.lib.lind_resolve(self.h, lam.real, lam.imag, _ptr(B), _ptr(X), tol, ctypes.byref(info))
        if rc and not (rc == LIND_ENOCONV and not raise_on_noconv):
            self._err(rc)
        d = info.as_dict()
        d["status"] = rc
        return X, d

    def implicit_euler(self, dt, steps, rho0, tol=1e-12, raise_on_noconv=True):
        """rho_steps of rho_{k+1} = (I - dt L)^{-1} rho_k (lind_ie).  Returns (rho, info)."""
        _check_mat(rho0, self.n, "rho0")
        out = self._new()
        info = LindInfo()
        rc = self.lib.lind_ie(self.h, float(dt), int(steps), _ptr(rho0), _ptr(out), tol, ctypes.byref(info))
        if rc and not (rc == LIND_ENOCONV and not raise_on_noconv):
            self._err(rc)
        d = info.as_dict()
        d["status"] = rc
        return out, d

    def factor(self, which):
        """Device tensors viewing the factorisation: 'G', 'T', 'Z', 'U', 'V' (n x n) or 's' (n)."""
        idx = {"G": 0, "T": 1, "Z": 2, "U": 3, "V": 4, "s": 5}[which]
        p = self.lib.lind_factor_ptr(self.h, idx)
        if not p:
            return None
        shape = (self.n,) if which == "s" else (self.n, self.n)
        out = self._new(*shape)
        nbytes = out.numel() * 16
        torch.cuda.current_stream(self.device).synchronize()
        _memcpy_d2d(out.data_ptr(), p, nbytes)
        return out


_hip = None


def _memcpy_d2d(dst, src, nbytes):
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    rc = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3)  # DeviceToDevice
    if rc:
        raise LindError(LIND_EDEVICE, f"hipMemcpy failed ({rc})")


class SteadyExpect(torch.autograd.Function):
    """J = Re Tr(O rho_inf(H, L)) with gradients from the adjoint solve (lind_steady_grad).

    forward(H, Ls, O, tol=1e-12, opts=None) -> 0-dim float64 tensor.  Gradients with respect to H
    and Ls follow PyTorch's convention for real losses of complex tensors (dJ/dRe + i dJ/dIm), so
    scalar physical parameters that build H and Ls by torch operations get their gradients by
    the chain rule.
    """

    @staticmethod
    def forward(ctx, H, Ls, O, tol=1e-12, opts=None):
        model = Lindblad(H.detach().contiguous(), Ls.detach().contiguous(), **(opts or {}))
        val, gH, gL, _, _ = model.steady_grad(O.detach().contiguous(), tol)
        model.close()
        ctx.save_for_backward(gH, gL)
        return torch.tensor(val, dtype=torch.float64, device=H.device)

    @staticmethod
    def backward(ctx, gout):
        gH, gL = ctx.saved_tensors
        g = gout.to(torch.complex128)
        return g * gH, g * gL, None, None, None


def steady_expectation(H, Ls, O, tol=1e-12, **opts):
    return SteadyExpect.apply(H, Ls, O, tol, opts)
