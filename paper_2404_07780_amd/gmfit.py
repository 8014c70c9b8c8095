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
ST_CONVERGED, ST_MAXITER, ST_STALLED, ST_NONFINITE, ST_TEAM_TIMEOUT = 0, 1, 2, 3, 4
SERSIC, EXPDISK, FERRER, KING, GAUSSIAN, MOFFAT, SKY, SKYPLANE = range(1, 9)

# exported symbols (one per declaration of include/gmfit.h)
SYMBOLS = ("gm_create", "gm_destroy", "gm_error_string", "gm_model_image", "gm_jacobian",
           "gm_default_guess", "gm_fit_batch", "gm_fit_batch_noalloc", "gm_param_errors", "gm_model_vjp", "gm_set_schedule",
           "gm_schedule_options", "gm_mlp_param_count", "gm_mlp_sync",
           "gm_mlp_forward", "gm_mlp_backward", "gm_mlp_adamw", "gm_mlp_train_step", "gm_mlp_gemm", "gm_features",
           "gm_proposal_targets", "gm_proposal_decode", "gm_fit_learned", "gm_synth_noise",
           "gm_plan_fit", "gm_plan_fit_learned", "gm_plan_launch", "gm_plan_elapsed", "gm_plan_destroy",
           "gm_bootstrap", "gm_fit_adam")


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


class gm_adam_opts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


class gm_fit_opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("lambda0", C.c_double), ("step_tol", C.c_double),
                ("active", C.c_void_p), ("proposal_max_iter", C.c_int32), ("err_out", C.c_void_p)]


class gm_schedule(C.Structure):
    _fields_ = [("plane_groups", C.c_int32), ("wg_per_cu", C.c_int32), ("team", C.c_int32),
                ("team_min_tiles", C.c_int32), ("team_wait_us", C.c_int32)]


class gm_mlp(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("hidden", C.c_int32), ("n_hidden", C.c_int32), ("out_dim", C.c_int32),
                ("n_out", C.c_int32), ("params", C.c_void_p), ("params_bf16", C.c_void_p), ("grad", C.c_void_p),
                ("adam_m", C.c_void_p), ("adam_v", C.c_void_p)]


class gm_adamw(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double)]


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
        L.gm_fit_batch_noalloc.argtypes = [v, p, p, p, v, v, v, v, v]
        L.gm_param_errors.argtypes = [v, p, p, v, v, v, v]
        L.gm_model_vjp.argtypes = [v, p, p, v, v, v, v]
        L.gm_set_schedule.argtypes = [v, p, i, p]
        L.gm_schedule_options.argtypes = [p, i, v, i, v]
        i64, u64, f, d = C.c_int64, C.c_uint64, C.c_float, C.c_double
        L.gm_mlp_param_count.argtypes = [p]
        L.gm_mlp_param_count.restype = i64
        L.gm_mlp_sync.argtypes = [v, p, v]
        L.gm_mlp_forward.argtypes = [v, p, i, v, i64, v, v]
        L.gm_mlp_backward.argtypes = [v, p, i, v, i64, v, v, v, v]
        L.gm_mlp_adamw.argtypes = [v, p, i64, p, v]
        L.gm_mlp_train_step.argtypes = [v, p, i, v, i64, v, v, i64, p, v, v]
        L.gm_mlp_gemm.argtypes = [v, i, i, i, i, v, i64, v, v, i64, v, v, i64, v]
        L.gm_features.argtypes = [v, p, p, v, i64, v, v]
        L.gm_proposal_targets.argtypes = [v, p, p, v, v, v, i, v]
        L.gm_proposal_decode.argtypes = [v, p, p, v, i, v, v, v, v]
        L.gm_fit_learned.argtypes = [v, p, p, p, p, v, v, v, v, v, v, v]
        L.gm_synth_noise.argtypes = [v, i, v, v, v, v, v, v, f, d, u64, i64, v, v, v, i, v]
        L.gm_plan_fit.argtypes = [v, p, p, p, v, v, v, v, v, v, i, C.POINTER(C.c_void_p)]
        L.gm_plan_fit_learned.argtypes = [v, p, p, p, p, v, v, v, v, v, v, i, C.POINTER(C.c_void_p)]
        L.gm_plan_launch.argtypes = [v, v]
        L.gm_bootstrap.argtypes = [v, p, p, p, v, i, u64, v, v, v, v, v]
        L.gm_plan_elapsed.argtypes = [v, v]
        L.gm_fit_adam.argtypes = [v, p, p, p, v, v, v, v]
        L.gm_plan_destroy.argtypes = [v]
        L.gm_plan_destroy.restype = None
        for name in ("gm_model_image", "gm_jacobian", "gm_default_guess", "gm_fit_batch", "gm_fit_batch_noalloc",
                     "gm_param_errors",
                     "gm_model_vjp", "gm_set_schedule", "gm_schedule_options", "gm_mlp_sync", "gm_mlp_forward", "gm_mlp_backward", "gm_mlp_adamw", "gm_mlp_train_step",
                     "gm_mlp_gemm", "gm_features", "gm_proposal_targets", "gm_proposal_decode", "gm_fit_learned",
                     "gm_synth_noise", "gm_plan_fit", "gm_plan_fit_learned", "gm_plan_launch",
                     "gm_plan_elapsed", "gm_bootstrap", "gm_fit_adam"):
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


def _err_ptr(err_out: Optional[torch.Tensor], batch: "Batch", model: "Model"):
    if err_out is None:
        return None
    if (err_out.dtype != torch.float64 or err_out.device != batch.device or not err_out.is_contiguous()
            or err_out.numel() != batch.n * model.p):
        raise ValueError("err_out: contiguous float64 device tensor of n_gal * p values")
    return err_out.data_ptr()


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


def gm_set_schedule(model: Model, psf_k: int, plane_groups: int = 0, wg_per_cu: int = 0, team: int = 0,
                    team_min_tiles: int = 0, team_wait_us: int = 0, ctx: Optional[Context] = None) -> None:
    """Schedule of the model's family at PSF side psf_k (0: every side without
    one): plane groups, persistent workgroups per CU, workgroups per fit
    (team: 0 automatic, 1 one, k > 1 up to k for fits of at least
    team_min_tiles tiles) and the bound of a team's waits (0: 20 s)."""
    ctx = ctx or context()
    m = model.c()
    sc = gm_schedule(int(plane_groups), int(wg_per_cu), int(team), int(team_min_tiles), int(team_wait_us))
    _check("gm_set_schedule", lib().gm_set_schedule(ctx.handle, C.byref(m), int(psf_k), C.byref(sc)))


def gm_schedule_options(model: Model, psf_k: int) -> List[int]:
    """Compiled plane-group counts of the model's family that fit at PSF side
    psf_k, preferred first."""
    m = model.c()
    buf = (C.c_int32 * 8)()
    n = C.c_int32()
    _check("gm_schedule_options", lib().gm_schedule_options(C.byref(m), int(psf_k), buf, 8, C.byref(n)))
    return [int(buf[i]) for i in range(min(n.value, 8))]


def gm_model_vjp(model: Model, batch: Batch, params, grad_image: torch.Tensor,
                 ctx: Optional[Context] = None) -> torch.Tensor:
    """sum over pixels of dM/dp * grad_image per galaxy: device [n][p] FP64."""
    ctx = ctx or context(batch.device.index)
    pr = _params_dev(params, batch, model.p)
    gi = grad_image.to(device=batch.device, dtype=torch.float32).contiguous()
    if gi.numel() != batch.npix:
        raise ValueError("grad_image must have the model image's size")
    grad = torch.empty(batch.n, model.p, dtype=torch.float64, device=batch.device)
    m, b = model.c(), batch.c()
    _check("gm_model_vjp", lib().gm_model_vjp(ctx.handle, C.byref(m), C.byref(b), _ptr(pr), _ptr(gi), _ptr(grad),
                                              _stream()))
    return grad


def gm_default_guess(model: Model, batch: Batch, ctx: Optional[Context] = None):
    ctx = ctx or context(batch.device.index)
    params = torch.zeros(batch.n, model.p, dtype=torch.float64, device=batch.device)
    mom = torch.zeros(batch.n, 6, dtype=torch.float64, device=batch.device)
    m, b = model.c(), batch.c()
    _check("gm_default_guess",
           lib().gm_default_guess(ctx.handle, C.byref(m), C.byref(b), _ptr(params), _ptr(mom), _stream()))
    return params, mom


def gm_fit_batch(model: Model, batch: Batch, params0, max_iter: int = 100, lambda0: float = 1e-3,
                 step_tol: float = 1e-4, ctx: Optional[Context] = None, out=None, active=None,
                 err_out: Optional[torch.Tensor] = None):
    """Returns (params, chi2, niter, status) as device tensors.  `out` may pass
    preallocated (params, chi2, niter, status); params is then overwritten with
    params0 first unless params0 is None.  `active` (device int32 [n]) skips
    the galaxies where it is 0.  `err_out` (device float64 [n, p]) receives
    the covariance errors at the fit."""
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
    o = gm_fit_opts(int(max_iter), float(lambda0), float(step_tol), None if active is None else active.data_ptr(), 0,
                    _err_ptr(err_out, batch, model))
    m, b = model.c(), batch.c()
    _check("gm_fit_batch", lib().gm_fit_batch(ctx.handle, C.byref(m), C.byref(b), C.byref(o), _ptr(params),
                                              _ptr(chi2), _ptr(niter), _ptr(status), _stream()))
    return params, chi2, niter, status


NOALLOC_MAX_GAL = 65536


def gm_fit_batch_noalloc(model: Model, batch: Batch, params: torch.Tensor, chi2: torch.Tensor,
                         niter: torch.Tensor, status: torch.Tensor, max_iter: int = 100, lambda0: float = 1e-3,
                         step_tol: float = 1e-4, ctx: Optional[Context] = None, active=None,
                         err_out: Optional[torch.Tensor] = None) -> None:
    """gm_fit_batch without any allocation, into the caller's device tensors:
    params (float64 [n, p], the start on entry, the fit on return), chi2
    (float64 [n]), niter and status (int32 [n])."""
    ctx = ctx or context(batch.device.index)
    for t, dt, shape in ((params, torch.float64, (batch.n, model.p)), (chi2, torch.float64, (batch.n,)),
                         (niter, torch.int32, (batch.n,)), (status, torch.int32, (batch.n,))):
        if t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous() or t.device != batch.device:
            raise ValueError("outputs must be contiguous device tensors of the batch's sizes")
    o = gm_fit_opts(int(max_iter), float(lambda0), float(step_tol), None if active is None else active.data_ptr(), 0,
                    _err_ptr(err_out, batch, model))
    m, b = model.c(), batch.c()
    _check("gm_fit_batch_noalloc", lib().gm_fit_batch_noalloc(ctx.handle, C.byref(m), C.byref(b), C.byref(o),
                                                              _ptr(params), _ptr(chi2), _ptr(niter), _ptr(status),
                                                              _stream()))


def gm_fit_adam(model: Model, batch: Batch, params0, steps: int = 1000, lr: float = 0.01, beta1: float = 0.9,
                beta2: float = 0.999, eps: float = 1e-8, ctx: Optional[Context] = None, out=None):
    """Gradient descent with Adam on chi^2 (the paper's fitter, Sec. 5.1).
    Returns (params, chi2, status) as device tensors; `out` may pass
    preallocated (params, chi2, status), params then overwritten with params0
    first unless params0 is None."""
    ctx = ctx or context(batch.device.index)
    if out is None:
        params = _params_dev(params0, batch, model.p).clone()
        chi2 = torch.empty(batch.n, dtype=torch.float64, device=batch.device)
        status = torch.empty(batch.n, dtype=torch.int32, device=batch.device)
    else:
        params, chi2, status = out
        if params0 is not None:
            params.copy_(_params_dev(params0, batch, model.p))
    o = gm_adam_opts(int(steps), float(lr), float(beta1), float(beta2), float(eps))
    m, b = model.c(), batch.c()
    _check("gm_fit_adam", lib().gm_fit_adam(ctx.handle, C.byref(m), C.byref(b), C.byref(o), _ptr(params),
                                            _ptr(chi2), _ptr(status), _stream()))
    return params, chi2, status


def gm_bootstrap(model: Model, batch: Batch, params, n_boot: int = 100, seed: int = 0, max_iter: int = 100,
                 lambda0: float = 1e-3, step_tol: float = 1e-4, want_replicas: bool = False,
                 ctx: Optional[Context] = None, out=None):
    """Poisson-bootstrap errors [n, p] (device); with want_replicas also the
    replica fits [n, n_boot, p], their status and trials [n, n_boot].  `out`
    may pass preallocated (err, rep_params, rep_status, rep_niter)."""
    ctx = ctx or context(batch.device.index)
    pr = _params_dev(params, batch, model.p)
    if out is not None:
        err, rp, rs, rn = out
    else:
        err = torch.empty(batch.n, model.p, dtype=torch.float64, device=batch.device)
        rp = rs = rn = None
        if want_replicas:
            rp = torch.empty(batch.n, n_boot, model.p, dtype=torch.float64, device=batch.device)
            rs = torch.empty(batch.n, n_boot, dtype=torch.int32, device=batch.device)
            rn = torch.empty(batch.n, n_boot, dtype=torch.int32, device=batch.device)
    o = gm_fit_opts(int(max_iter), float(lambda0), float(step_tol), None, 0, None)
    m, b = model.c(), batch.c()
    _check("gm_bootstrap", lib().gm_bootstrap(ctx.handle, C.byref(m), C.byref(b), C.byref(o), _ptr(pr), int(n_boot),
                                              int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(err), _ptr(rp), _ptr(rs),
                                              _ptr(rn), _stream()))
    return (err, rp, rs, rn) if (want_replicas or out is not None) else err


def gm_param_errors(model: Model, batch: Batch, params, want_cov: bool = False, ctx: Optional[Context] = None):
    ctx = ctx or context(batch.device.index)
    pr = _params_dev(params, batch, model.p)
    err = torch.empty(batch.n, model.p, dtype=torch.float64, device=batch.device)
    cov = torch.empty(batch.n, model.p, model.p, dtype=torch.float64, device=batch.device) if want_cov else None
    m, b = model.c(), batch.c()
    _check("gm_param_errors",
           lib().gm_param_errors(ctx.handle, C.byref(m), C.byref(b), _ptr(pr), _ptr(err), _ptr(cov), _stream()))
    return (err, cov) if want_cov else err


# ---------------------------------------------------------------- learned proposal
class MLP:
    """Network parameters on the device: FP32 master, BF16 copy, gradient and
    AdamW moments (flat vectors, layout of include/gmfit.h)."""

    def __init__(self, params, in_dim: int = 1056, hidden: int = 512, n_hidden: int = 3, out_dim: int = 16,
                 n_out: int = 7, device=None, train: bool = True):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.dims = (in_dim, hidden, n_hidden, out_dim, n_out)
        self.device = dev
        probe = gm_mlp(in_dim, hidden, n_hidden, out_dim, n_out)
        cnt = lib().gm_mlp_param_count(C.byref(probe))
        if cnt < 0:
            raise ValueError("invalid network sizes")
        t = params if isinstance(params, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(params, np.float32))
        if t.numel() != cnt:
            raise ValueError(f"expected {cnt} parameters, got {t.numel()}")
        self.params = t.to(device=dev, dtype=torch.float32).contiguous().clone()
        self.params_bf16 = torch.empty(cnt, dtype=torch.bfloat16, device=dev)
        self.grad = torch.zeros(cnt, dtype=torch.float32, device=dev) if train else None
        self.adam_m = torch.zeros(cnt, dtype=torch.float32, device=dev) if train else None
        self.adam_v = torch.zeros(cnt, dtype=torch.float32, device=dev) if train else None
        self.step = 0
        gm_mlp_sync(self)

    def c(self) -> gm_mlp:
        m = gm_mlp(*self.dims)
        m.params = self.params.data_ptr()
        m.params_bf16 = self.params_bf16.data_ptr()
        for name in ("grad", "adam_m", "adam_v"):
            t = getattr(self, name)
            setattr(m, name, None if t is None else t.data_ptr())
        return m


def _ctx_for(device, ctx):
    return ctx or context(device.index)


def _bf16_rows(x: torch.Tensor, min_cols: int) -> torch.Tensor:
    if x.dtype != torch.bfloat16 or x.dim() != 2 or x.shape[1] < min_cols or x.stride(1) != 1:
        raise ValueError("x must be a 2-D BF16 tensor with unit column stride")
    return x


def gm_mlp_sync(mlp: MLP, ctx: Optional[Context] = None) -> None:
    ctx = _ctx_for(mlp.device, ctx)
    m = mlp.c()
    _check("gm_mlp_sync", lib().gm_mlp_sync(ctx.handle, C.byref(m), _stream()))


def gm_mlp_forward(mlp: MLP, x: torch.Tensor, ctx: Optional[Context] = None) -> torch.Tensor:
    ctx = _ctx_for(mlp.device, ctx)
    x = _bf16_rows(x, mlp.dims[0])
    out = torch.empty(x.shape[0], mlp.dims[3], dtype=torch.float32, device=mlp.device)
    m = mlp.c()
    _check("gm_mlp_forward", lib().gm_mlp_forward(ctx.handle, C.byref(m), x.shape[0], _ptr(x), x.stride(0),
                                                  _ptr(out), _stream()))
    return out


def gm_mlp_backward(mlp: MLP, x: torch.Tensor, targets: torch.Tensor, rows: Optional[torch.Tensor] = None,
                    n: Optional[int] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Gradient into mlp.grad; returns the loss (device FP64 scalar)."""
    ctx = _ctx_for(mlp.device, ctx)
    x = _bf16_rows(x, mlp.dims[0])
    n = int(rows.numel() if rows is not None else (x.shape[0] if n is None else n))
    loss = torch.empty((), dtype=torch.float64, device=mlp.device)
    m = mlp.c()
    _check("gm_mlp_backward", lib().gm_mlp_backward(ctx.handle, C.byref(m), n, _ptr(x), x.stride(0), _ptr(rows),
                                                    _ptr(targets), _ptr(loss), _stream()))
    return loss


GEMM_NT, GEMM_NN, GEMM_TN = 0, 1, 2


def gm_mlp_gemm(op: int, a: torch.Tensor, b: torch.Tensor, a_rows: Optional[torch.Tensor] = None,
                b_rows: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """FP32 product of two device BF16 matrices by the dense layers' kernels:
    NT: a [m][k] (rows gathered by a_rows), b [n][k] -> a b^T; NN: a [m][k]
    (a_rows), b [k][n] -> a b; TN: a [k][m], b [k][n] (rows gathered by b_rows)
    -> a^T b."""
    for t in (a, b):
        if t.dtype != torch.bfloat16 or t.dim() != 2 or t.stride(1) != 1:
            raise ValueError("operands must be 2-D BF16 tensors with unit column stride")
    if op == GEMM_NT:
        m, k, n = (a_rows.numel() if a_rows is not None else a.shape[0]), a.shape[1], b.shape[0]
    elif op == GEMM_NN:
        m, k, n = (a_rows.numel() if a_rows is not None else a.shape[0]), a.shape[1], b.shape[1]
    else:
        k, m, n = (b_rows.numel() if b_rows is not None else b.shape[0]), a.shape[1], b.shape[1]
    ctx = _ctx_for(a.device, ctx)
    c = torch.empty(m, n, dtype=torch.float32, device=a.device)
    _check("gm_mlp_gemm", lib().gm_mlp_gemm(ctx.handle, op, m, n, k, _ptr(a), a.stride(0), _ptr(a_rows), _ptr(b),
                                            b.stride(0), _ptr(b_rows), _ptr(c), c.stride(0), _stream()))
    return c


def gm_mlp_adamw(mlp: MLP, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                 weight_decay: float = 0.0, ctx: Optional[Context] = None) -> None:
    ctx = _ctx_for(mlp.device, ctx)
    mlp.step += 1
    o = gm_adamw(lr, beta1, beta2, eps, weight_decay)
    m = mlp.c()
    _check("gm_mlp_adamw", lib().gm_mlp_adamw(ctx.handle, C.byref(m), mlp.step, C.byref(o), _stream()))


def gm_mlp_train_step(mlp: MLP, x: torch.Tensor, targets: torch.Tensor, rows: Optional[torch.Tensor], lr: float,
                      beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, weight_decay: float = 0.0,
                      loss: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    ctx = _ctx_for(mlp.device, ctx)
    x = _bf16_rows(x, mlp.dims[0])
    n = int(rows.numel() if rows is not None else x.shape[0])
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=mlp.device)
    mlp.step += 1
    o = gm_adamw(lr, beta1, beta2, eps, weight_decay)
    m = mlp.c()
    _check("gm_mlp_train_step", lib().gm_mlp_train_step(ctx.handle, C.byref(m), n, _ptr(x), x.stride(0),
                                                        _ptr(rows), _ptr(targets), mlp.step, C.byref(o),
                                                        _ptr(loss), _stream()))
    return loss


def gm_features(model: Model, batch: Batch, ctx: Optional[Context] = None, ldx: int = 1056):
    """(features [n][ldx] BF16, moments [n][8] FP64) as device tensors."""
    ctx = _ctx_for(batch.device, ctx)
    x = torch.zeros(batch.n, ldx, dtype=torch.bfloat16, device=batch.device)
    mom = torch.empty(batch.n, 8, dtype=torch.float64, device=batch.device)
    m, b = model.c(), batch.c()
    _check("gm_features", lib().gm_features(ctx.handle, C.byref(m), C.byref(b), _ptr(x), ldx, _ptr(mom), _stream()))
    return x, mom


def gm_proposal_targets(model: Model, batch: Batch, truth, moments: torch.Tensor, out_dim: int = 16,
                        ctx: Optional[Context] = None) -> torch.Tensor:
    ctx = _ctx_for(batch.device, ctx)
    tr = _params_dev(truth, batch, model.p)
    t = torch.empty(batch.n, out_dim, dtype=torch.float32, device=batch.device)
    m, b = model.c(), batch.c()
    _check("gm_proposal_targets", lib().gm_proposal_targets(ctx.handle, C.byref(m), C.byref(b), _ptr(tr),
                                                            _ptr(moments), _ptr(t), out_dim, _stream()))
    return t


def gm_proposal_decode(model: Model, batch: Batch, out: torch.Tensor, moments: torch.Tensor,
                       ctx: Optional[Context] = None):
    ctx = _ctx_for(batch.device, ctx)
    params = torch.zeros(batch.n, model.p, dtype=torch.float64, device=batch.device)
    valid = torch.empty(batch.n, dtype=torch.int32, device=batch.device)
    m, b = model.c(), batch.c()
    _check("gm_proposal_decode", lib().gm_proposal_decode(ctx.handle, C.byref(m), C.byref(b), _ptr(out),
                                                          out.shape[1], _ptr(moments), _ptr(params), _ptr(valid),
                                                          _stream()))
    return params, valid


def gm_fit_learned(model: Model, batch: Batch, mlp: MLP, max_iter: int = 100, lambda0: float = 1e-3,
                   step_tol: float = 1e-4, proposal_max_iter: int = 20, ctx: Optional[Context] = None, out=None,
                   events=None, err_out: Optional[torch.Tensor] = None):
    """(params, chi2, niter, status, fallback) as device tensors.  The LM from the
    learned start gets proposal_max_iter trials (0: max_iter) before the
    fallback.  events: four recorded torch.cuda.Event objects that the library
    re-records around its two LM launches.  err_out (device float64 [n, p])
    receives the covariance errors at the fit."""
    ctx = _ctx_for(batch.device, ctx)
    if out is None:
        params = torch.zeros(batch.n, model.p, dtype=torch.float64, device=batch.device)
        chi2 = torch.empty(batch.n, dtype=torch.float64, device=batch.device)
        niter = torch.empty(batch.n, dtype=torch.int32, device=batch.device)
        status = torch.empty(batch.n, dtype=torch.int32, device=batch.device)
        fallback = torch.empty(batch.n, dtype=torch.int32, device=batch.device)
    else:
        params, chi2, niter, status, fallback = out
    o = gm_fit_opts(int(max_iter), float(lambda0), float(step_tol), None, int(proposal_max_iter),
                    _err_ptr(err_out, batch, model))
    m, b, ml = model.c(), batch.c(), mlp.c()
    ev = _events4(events)
    _check("gm_fit_learned", lib().gm_fit_learned(ctx.handle, C.byref(m), C.byref(b), C.byref(ml), C.byref(o),
                                                  _ptr(params), _ptr(chi2), _ptr(niter), _ptr(status),
                                                  _ptr(fallback), ev, _stream()))
    return params, chi2, niter, status, fallback


def _events4(events):
    if events is None:
        return None
    if len(events) != 4 or any(int(e.cuda_event) == 0 for e in events):
        raise ValueError("events: four torch.cuda.Event objects, each recorded once")
    return (C.c_void_p * 4)(*[int(e.cuda_event) for e in events])


class Plan:
    """A captured call sequence (gm_plan_fit / gm_plan_fit_learned): launch()
    replays its graph on the current stream.  The plan holds the batch, the
    inputs and its output tensors (attributes params, chi2, niter, status,
    fallback, err) so that every pointer baked into the graph stays valid."""

    def __init__(self, handle, device, keep, **outputs):
        self._h = handle
        self.device = device
        self._keep = keep
        for k, t in outputs.items():
            setattr(self, k, t)

    def launch(self) -> None:
        if not self._h:
            raise RuntimeError("plan destroyed")
        _check("gm_plan_launch", lib().gm_plan_launch(self._h, _stream()))

    def elapsed(self) -> List[float]:
        """Milliseconds between the plan's four timing events in its latest
        launch (waits for it); plans made with timing=True."""
        ms = (C.c_float * 3)()
        _check("gm_plan_elapsed", lib().gm_plan_elapsed(self._h, ms))
        return [float(v) for v in ms]

    def close(self) -> None:
        if self._h:
            lib().gm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _fit_outputs(model: Model, batch: Batch, errors: bool, fallback: bool):
    dev = batch.device
    out = dict(params=torch.zeros(batch.n, model.p, dtype=torch.float64, device=dev),
               chi2=torch.empty(batch.n, dtype=torch.float64, device=dev),
               niter=torch.empty(batch.n, dtype=torch.int32, device=dev),
               status=torch.empty(batch.n, dtype=torch.int32, device=dev),
               err=torch.empty(batch.n, model.p, dtype=torch.float64, device=dev) if errors else None)
    if fallback:
        out["fallback"] = torch.empty(batch.n, dtype=torch.int32, device=dev)
    return out


def gm_plan_fit(model: Model, batch: Batch, start=None, errors: bool = True, max_iter: int = 100,
                lambda0: float = 1e-3, step_tol: float = 1e-4, active=None, timing: bool = False,
                ctx: Optional[Context] = None) -> Plan:
    """Capture start (None: the moment-based guess) -> LM -> (errors) on this
    batch.  Each launch() refits from `start`: a contiguous float64 device
    tensor [n, p] is used in place (its contents may change between
    launches); anything else is copied once."""
    ctx = _ctx_for(batch.device, ctx)
    st = None if start is None else _params_dev(start, batch, model.p).contiguous()
    out = _fit_outputs(model, batch, errors, False)
    o = gm_fit_opts(int(max_iter), float(lambda0), float(step_tol), None if active is None else active.data_ptr(), 0)
    m, b = model.c(), batch.c()
    h = C.c_void_p()
    _check("gm_plan_fit", lib().gm_plan_fit(ctx.handle, C.byref(m), C.byref(b), C.byref(o), _ptr(st),
                                            _ptr(out["params"]), _ptr(out["chi2"]), _ptr(out["niter"]),
                                            _ptr(out["status"]), _ptr(out["err"]), int(bool(timing)), C.byref(h)))
    return Plan(h, batch.device, (ctx, batch, st, active), **out)


def gm_plan_fit_learned(model: Model, batch: Batch, mlp: "MLP", errors: bool = True, max_iter: int = 100,
                        lambda0: float = 1e-3, step_tol: float = 1e-4, proposal_max_iter: int = 20,
                        timing: bool = False, ctx: Optional[Context] = None) -> Plan:
    """Capture gm_fit_learned -> (errors) on this batch; the network's weights
    are read at each launch."""
    ctx = _ctx_for(batch.device, ctx)
    out = _fit_outputs(model, batch, errors, True)
    o = gm_fit_opts(int(max_iter), float(lambda0), float(step_tol), None, int(proposal_max_iter))
    m, b, ml = model.c(), batch.c(), mlp.c()
    h = C.c_void_p()
    _check("gm_plan_fit_learned",
           lib().gm_plan_fit_learned(ctx.handle, C.byref(m), C.byref(b), C.byref(ml), C.byref(o), _ptr(out["params"]),
                                     _ptr(out["chi2"]), _ptr(out["niter"]), _ptr(out["status"]),
                                     _ptr(out["fallback"]), _ptr(out["err"]), int(bool(timing)), C.byref(h)))
    return Plan(h, batch.device, (ctx, batch, mlp), **out)


def gm_synth_noise(h, w, img_off, unit: torch.Tensor, snr: torch.Tensor, sky: torch.Tensor, sigma: float,
                   seed: int, first_index: int = 0, m0: float = 22.5, mag_out: Optional[torch.Tensor] = None,
                   mag_stride: int = 1, ctx: Optional[Context] = None):
    """(data, sigma map) device FP32 images; mag_out[g * mag_stride] gets the
    magnitude that gives each galaxy its peak SNR."""
    ctx = _ctx_for(unit.device, ctx)
    h = np.ascontiguousarray(h, np.int32)
    w = np.ascontiguousarray(w, np.int32)
    img_off = np.ascontiguousarray(img_off, np.int64)
    data = torch.empty_like(unit)
    sig = torch.empty_like(unit)
    _check("gm_synth_noise", lib().gm_synth_noise(ctx.handle, len(h), h.ctypes.data, w.ctypes.data,
                                                  img_off.ctypes.data, _ptr(unit), _ptr(snr), _ptr(sky),
                                                  float(sigma), float(m0), int(seed), int(first_index), _ptr(data),
                                                  _ptr(sig), _ptr(mag_out), int(mag_stride), _stream()))
    return data, sig
