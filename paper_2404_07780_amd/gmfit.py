"""Python binding of libgmfit.so (C ABI in include/gmfit.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device arrays are torch tensors on the HIP device (torch supplies
device memory and the current stream); size metadata stays in numpy on the
host, as the ABI requires.  There is no CPU fallback: if the library is not
built, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libgmfit.so")

GM_OK, GM_EINVAL, GM_EHIP, GM_ENOMEM, GM_EUNSUPPORTED = 0, -1, -2, -3, -4
ST_CONVERGED, ST_MAXITER, ST_STALLED, ST_NONFINITE = 0, 1, 2, 3
SERSIC, EXPDISK, FERRER, KING, GAUSSIAN, MOFFAT, SKY = range(1, 8)

# exported symbols (one per declaration of include/gmfit.h)
SYMBOLS = ("gm_create", "gm_destroy", "gm_error_string", "gm_model_image", "gm_jacobian",
           "gm_default_guess", "gm_fit_batch", "gm_param_errors")


class GmError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn}: {error_string(code)} ({code})")
        self.code = code


class gm_component(C.Structure):
    _fields_ = [("type", C.c_int32), ("convolve", C.c_int32), ("param_index", C.c_int32 * 8),
                ("fixed", C.c_double * 8)]


class gm_model(C.Structure):
    _fields_ = [("n_comp", C.c_int32), ("comp", gm_component * 4), ("p", C.c_int32), ("m0", C.c_double),
                ("oversample", C.c_int32), ("os_window", C.c_int32)]


class gm_batch(C.Structure):
    _fields_ = [("n_gal", C.c_int32), ("h", C.c_void_p), ("w", C.c_void_p), ("img_off", C.c_void_p),
                ("psf_k", C.c_void_p), ("psf_off", C.c_void_p), ("data", C.c_void_p), ("sigma", C.c_void_p),
                ("omega", C.c_void_p), ("psf", C.c_void_p)]


class gm_fit_opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("lambda0", C.c_double), ("step_tol", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load libgmfit.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"libgmfit.so not built ({_LIB_PATH}); run paper_2404_07780_amd/build.py")
        L = C.CDLL(_LIB_PATH)
        v, i, p = C.c_void_p, C.c_int, C.c_void_p
        L.gm_create.argtypes = [C.POINTER(C.c_void_p), i]
        L.gm_create.restype = i
        L.gm_destroy.argtypes = [v]
        L.gm_destroy.restype = None
        L.gm_error_string.argtypes = [i]
        L.gm_error_string.restype = C.c_char_p
        L.gm_model_image.argtypes = [v, p, p, v, v, v]
        L.gm_jacobian.argtypes = [v, p, p, v, v, v]
        L.gm_default_guess.argtypes = [v, p, p, v, v, v]
        L.gm_fit_batch.argtypes = [v, p, p, p, v, v, v, v, v]
        L.gm_param_errors.argtypes = [v, p, p, v, v, v, v]
        for name in ("gm_model_image", "gm_jacobian", "gm_default_guess", "gm_fit_batch", "gm_param_errors"):
            getattr(L, name).restype = i
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().gm_error_string(int(code)).decode()


def _check(fn: str, rc: int) -> None:
    if rc != GM_OK:
        raise GmError(fn, rc)


# ---------------------------------------------------------------- descriptions
@dataclass
class Component:
    type: int
    convolve: bool
    param_index: Sequence[int]
    fixed: Sequence[float] = ()


@dataclass
class Model:
    comps: List[Component]
    p: int
    m0: float = 22.5
    oversample: int = 10
    os_window: int = 5

    @staticmethod
    def from_spec(spec: dict, **kw) -> "Model":
        return Model([Component(t, bool(c), idx, fx) for t, c, idx, fx in spec["comps"]], spec["p"], **kw)

    def c(self) -> gm_model:
        m = gm_model()
        m.n_comp = len(self.comps)
        for k, cp in enumerate(self.comps):
            m.comp[k].type = cp.type
            m.comp[k].convolve = 1 if cp.convolve else 0
            for s in range(8):
                m.comp[k].param_index[s] = cp.param_index[s] if s < len(cp.param_index) else -1
                m.comp[k].fixed[s] = cp.fixed[s] if s < len(cp.fixed) else 0.0
        m.p = self.p
        m.m0 = self.m0
        m.oversample = self.oversample
        m.os_window = self.os_window
        return m


class Batch:
    """A ragged batch resident on the device, plus its host-side size metadata."""

    def __init__(self, h, w, img_off, psf_k, psf_off, data, sigma, psf, omega=None, device=None):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.h = np.ascontiguousarray(h, np.int32)
        self.w = np.ascontiguousarray(w, np.int32)
        self.img_off = np.ascontiguousarray(img_off, np.int64)
        self.psf_k = np.ascontiguousarray(psf_k, np.int32)
        self.psf_off = np.ascontiguousarray(psf_off, np.int64)

        def dev_t(a, dt):
            if a is None:
                return None
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            return t.to(device=dev, dtype=dt).contiguous()

        self.data = dev_t(data, torch.float32)
        self.sigma = dev_t(sigma, torch.float32)
        self.psf = dev_t(psf, torch.float32)
        self.omega = dev_t(omega, torch.uint8)
        self.device = dev

    @property
    def n(self) -> int:
        return len(self.h)

    @property
    def npix(self) -> int:
        return int(self.img_off[-1] + int(self.h[-1]) * int(self.w[-1])) if self.n else 0

    def c(self) -> gm_batch:
        b = gm_batch()
        b.n_gal = self.n
        b.h = self.h.ctypes.data
        b.w = self.w.ctypes.data
        b.img_off = self.img_off.ctypes.data
        b.psf_k = self.psf_k.ctypes.data
        b.psf_off = self.psf_off.ctypes.data
        b.data = self.data.data_ptr() if self.data is not None else None
        b.sigma = self.sigma.data_ptr() if self.sigma is not None else None
        b.omega = self.omega.data_ptr() if self.omega is not None else None
        b.psf = self.psf.data_ptr() if self.psf is not None else None
        return b


class Context:
    """gm_ctx on one HIP device."""

    def __init__(self, device: Optional[int] = None):
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        _check("gm_create", lib().gm_create(C.byref(h), self.device))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().gm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def context(device: Optional[int] = None) -> Context:
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _default_ctx:
        _default_ctx[d] = Context(d)
    return _default_ctx[d]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _params_dev(params, batch: Batch, p: int) -> torch.Tensor:
    t = params if isinstance(params, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(params, np.float64))
    t = t.to(device=batch.device, dtype=torch.float64).contiguous()
    if t.numel() != batch.n * p:
        raise ValueError(f"params must hold n_gal * p = {batch.n * p} values")
    return t.view(batch.n, p)


# ---------------------------------------------------------------- entry points
def gm_model_image(model: Model, batch: Batch, params, ctx: Optional[Context] = None) -> torch.Tensor:
    ctx = ctx or context(batch.device.index)
    pr = _params_dev(params, batch, model.p)
    out = torch.empty(batch.npix, dtype=torch.float32, device=batch.device)
    m, b = model.c(), batch.c()
    _check("gm_model_image", lib().gm_model_image(ctx.handle, C.byref(m), C.byref(b), _ptr(pr), _ptr(out), _stream()))
    return out


def gm_jacobian(model: Model, batch: Batch, params, ctx: Optional[Context] = None) -> torch.Tensor:
    """Concatenated per-galaxy [p][h][w] blocks (galaxy g at p * img_off[g])."""
    ctx = ctx or context(batch.device.index)
    pr = _params_dev(params, batch, model.p)
    out = torch.empty(batch.npix * model.p, dtype=torch.float32, device=batch.device)
    m, b = model.c(), batch.c()
    _check("gm_jacobian", lib().gm_jacobian(ctx.handle, C.byref(m), C.byref(b), _ptr(pr), _ptr(out), _stream()))
    return out


def gm_default_guess(model: Model, batch: Batch, ctx: Optional[Context] = None):
    ctx = ctx or context(batch.device.index)
    params = torch.zeros(batch.n, model.p, dtype=torch.float64, device=batch.device)
    mom = torch.zeros(batch.n, 6, dtype=torch.float64, device=batch.device)
    m, b = model.c(), batch.c()
    _check("gm_default_guess",
           lib().gm_default_guess(ctx.handle, C.byref(m), C.byref(b), _ptr(params), _ptr(mom), _stream()))
    return params, mom


def gm_fit_batch(model: Model, batch: Batch, params0, max_iter: int = 100, lambda0: float = 1e-3,
                 step_tol: float = 1e-4, ctx: Optional[Context] = None, out=None):
    """Returns (params, chi2, niter, status) as device tensors.  `out` may pass
    preallocated (params, chi2, niter, status); params is then overwritten with
    params0 first unless params0 is None."""
    ctx = ctx or context(batch.device.index)
    if out is None:
        params = _params_dev(params0, batch, model.p).clone()
        chi2 = torch.empty(batch.n, dtype=torch.float64, device=batch.device)
        niter = torch.empty(batch.n, dtype=torch.int32, device=batch.device)
        status = torch.empty(batch.n, dtype=torch.int32, device=batch.device)
    else:
        params, chi2, niter, status = out
        if params0 is not None:
            params.copy_(_params_dev(params0, batch, model.p))
    o = gm_fit_opts(int(max_iter), float(lambda0), float(step_tol))
    m, b = model.c(), batch.c()
    _check("gm_fit_batch", lib().gm_fit_batch(ctx.handle, C.byref(m), C.byref(b), C.byref(o), _ptr(params),
                                              _ptr(chi2), _ptr(niter), _ptr(status), _stream()))
    return params, chi2, niter, status


def gm_param_errors(model: Model, batch: Batch, params, want_cov: bool = False, ctx: Optional[Context] = None):
    ctx = ctx or context(batch.device.index)
    pr = _params_dev(params, batch, model.p)
    err = torch.empty(batch.n, model.p, dtype=torch.float64, device=batch.device)
    cov = torch.empty(batch.n, model.p, model.p, dtype=torch.float64, device=batch.device) if want_cov else None
    m, b = model.c(), batch.c()
    _check("gm_param_errors",
           lib().gm_param_errors(ctx.handle, C.byref(m), C.byref(b), _ptr(pr), _ptr(err), _ptr(cov), _stream()))
    return (err, cov) if want_cov else err
