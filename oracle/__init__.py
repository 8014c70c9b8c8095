"""FP64 CPU oracle for batched Levenberg-Marquardt galaxy-profile fitting.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
CPU-baseline leg of the benchmark may load it; the product package never
imports it.  It shares no code with the HIP path: the arithmetic lives in
``gm_oracle.c`` (plain C, double precision), this module only marshals
numpy arrays through ctypes.

Parameter vectors are in natural units: pixels for centres and scales,
magnitudes, degrees for position angles, counts per pixel for sky.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SERSIC, EXPDISK, FERRER, KING, GAUSSIAN, MOFFAT, SKY, SKYPLANE = range(1, 9)
ST_CONVERGED, ST_MAXITER, ST_STALLED, ST_NONFINITE = 0, 1, 2, 3
MAX_COMP, MAX_SLOTS, MAX_P = 4, 8, 16

# natural slots of each profile type
SLOTS = {
    SERSIC: ("x0", "y0", "mag", "re", "n", "q", "pa", "box"),
    EXPDISK: ("x0", "y0", "mag", "rs", "q", "pa"),
    FERRER: ("x0", "y0", "mag", "rout", "q", "pa", "a", "b"),
    KING: ("x0", "y0", "I0", "rc", "rt", "q", "pa", "alpha"),
    GAUSSIAN: ("x0", "y0", "I0", "fwhm", "q", "pa"),
    MOFFAT: ("x0", "y0", "mag", "fwhm", "q", "pa", "beta"),
    SKY: ("sky",),
    SKYPLANE: ("sky", "kx", "ky"),
}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C11, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Comp(C.Structure):
    _fields_ = [
        ("type", C.c_int32),
        ("convolve", C.c_int32),
        ("idx", C.c_int32 * MAX_SLOTS),
        ("fixed", C.c_double * MAX_SLOTS),
    ]


class _Model(C.Structure):
    _fields_ = [
        ("ncomp", C.c_int32),
        ("comp", _Comp * MAX_COMP),
        ("p", C.c_int32),
        ("m0", C.c_double),
        ("oversample", C.c_int32),
        ("os_window", C.c_int32),
    ]


class _Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("lambda0", C.c_double), ("step_tol", C.c_double)]


class _AdamOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


@dataclass
class Comp:
    type: int
    convolve: bool
    idx: Sequence[int]
    fixed: Sequence[float] = ()


@dataclass
class Model:
    comps: List[Comp]
    p: int
    m0: float = 22.5
    oversample: int = 10
    os_window: int = 5

    def c(self) -> _Model:
        m = _Model()
        m.ncomp = len(self.comps)
        for i, cp in enumerate(self.comps):
            m.comp[i].type = cp.type
            m.comp[i].convolve = 1 if cp.convolve else 0
            for s in range(MAX_SLOTS):
                m.comp[i].idx[s] = cp.idx[s] if s < len(cp.idx) else -1
                m.comp[i].fixed[s] = cp.fixed[s] if s < len(cp.fixed) else 0.0
        m.p = self.p
        m.m0 = self.m0
        m.oversample = self.oversample
        m.os_window = self.os_window
        return m


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        d, i, p = C.c_double, C.c_int, C.c_void_p
        for name in ("orc_digamma", "orc_sersic_b", "orc_sersic_db"):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = [d]
        for name in ("orc_gammainc_p", "orc_dgammainc_p_da"):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = [d, d]
        L.orc_validate.argtypes = [p]
        L.orc_convolve.argtypes = [i, i, p, i, p, p]
        L.orc_convolve.restype = None
        L.orc_canonicalise.argtypes = [p, p]
        L.orc_canonicalise.restype = None
        L.orc_profile_point.argtypes = [p, i, p, d, d, p, p]
        L.orc_model_image.argtypes = [p, i, i, p, i, p, p]
        L.orc_jacobian.argtypes = [p, i, i, p, i, p, p]
        L.orc_fit.argtypes = [p, i, i, p, p, p, p, i, p, p, p, p, p]
        L.orc_param_errors.argtypes = [p, i, i, p, p, p, p, i, p, p, p]
        L.orc_default_guess.argtypes = [p, i, i, p, p, p, p, p]
        L.orc_moments.argtypes = [i, i, p, p, p, d, p]
        L.orc_moments.restype = None
        L.orc_fit_batch.argtypes = [p, i, p, p, p, p, p, p, p, p, p, p, p, p, p, p, i]
        L.orc_fit_adam.argtypes = [p, i, i, p, p, p, p, i, p, p, p, p]
        L.orc_fit_adam_batch.argtypes = [p, i, p, p, p, p, p, p, p, p, p, p, p, p, p, i]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---- special functions --------------------------------------------------
def digamma(x: float) -> float:
    return lib().orc_digamma(float(x))


def gammainc_p(a: float, x: float) -> float:
    return lib().orc_gammainc_p(float(a), float(x))


def dgammainc_p_da(a: float, x: float) -> float:
    return lib().orc_dgammainc_p_da(float(a), float(x))


def sersic_b(n: float) -> float:
    return lib().orc_sersic_b(float(n))


def sersic_db(n: float) -> float:
    return lib().orc_sersic_db(float(n))


# ---- images --------------------------------------------------------------
def profile_point(model: Model, comp: int, params, x: float, y: float):
    """(I, dI/du per natural slot) of one component at the point (x, y)."""
    params = _f64(params)
    I = C.c_double()
    dI = np.zeros(MAX_SLOTS)
    mc = model.c()
    rc = lib().orc_profile_point(C.byref(mc), comp, _ptr(params), float(x), float(y), C.byref(I), _ptr(dI))
    if rc != 0:
        raise ValueError(f"orc_profile_point failed ({rc})")
    return I.value, dI


def convolve(img: np.ndarray, psf: np.ndarray) -> np.ndarray:
    img = _f64(img)
    psf = _f64(psf)
    out = np.empty_like(img)
    lib().orc_convolve(img.shape[0], img.shape[1], _ptr(img), psf.shape[0], _ptr(psf), _ptr(out))
    return out


def model_image(model: Model, h: int, w: int, psf: np.ndarray, params) -> np.ndarray:
    psf = _f32(psf)
    params = _f64(params)
    out = np.empty((h, w), np.float64)
    mc = model.c()
    rc = lib().orc_model_image(C.byref(mc), h, w, _ptr(psf), psf.shape[0], _ptr(params), _ptr(out))
    if rc != 0:
        raise ValueError(f"orc_model_image failed ({rc})")
    return out


def jacobian(model: Model, h: int, w: int, psf: np.ndarray, params) -> np.ndarray:
    """dM/dp for every column p of the natural parameter vector: [p][h][w]."""
    psf = _f32(psf)
    params = _f64(params)
    out = np.empty((model.p, h, w), np.float64)
    mc = model.c()
    rc = lib().orc_jacobian(C.byref(mc), h, w, _ptr(psf), psf.shape[0], _ptr(params), _ptr(out))
    if rc != 0:
        raise ValueError(f"orc_jacobian failed ({rc})")
    return out


def canonicalise(model: Model, params) -> np.ndarray:
    params = _f64(params).copy()
    mc = model.c()
    lib().orc_canonicalise(C.byref(mc), _ptr(params))
    return params


def fit(model: Model, data, sigma, psf, params0, omega=None, max_iter=100, lambda0=1e-3, step_tol=1e-4):
    """LM fit of one galaxy; returns (params, chi2, niter, status)."""
    data = _f32(data)
    sigma = _f32(sigma)
    psf = _f32(psf)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.uint8)
    params = _f64(params0).copy()
    chi2 = C.c_double()
    nit = C.c_int()
    st = C.c_int()
    o = _Opts(max_iter, lambda0, step_tol)
    mc = model.c()
    rc = lib().orc_fit(C.byref(mc), data.shape[0], data.shape[1], _ptr(data), _ptr(sigma), _ptr(om),
                       _ptr(psf), psf.shape[0], C.byref(o), _ptr(params), C.byref(chi2), C.byref(nit),
                       C.byref(st))
    if rc != 0:
        raise ValueError(f"orc_fit failed ({rc})")
    return params, chi2.value, nit.value, st.value


def fit_adam(model: Model, data, sigma, psf, params0, omega=None, steps=1000, lr=0.01, beta1=0.9,
             beta2=0.999, eps=1e-8):
    """Gradient descent with Adam on chi^2 (Sec. 5.1), one galaxy; returns
    (params, chi2, status)."""
    data = _f32(data)
    sigma = _f32(sigma)
    psf = _f32(psf)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.uint8)
    params = _f64(params0).copy()
    chi2 = C.c_double()
    st = C.c_int()
    o = _AdamOpts(steps, lr, beta1, beta2, eps)
    mc = model.c()
    rc = lib().orc_fit_adam(C.byref(mc), data.shape[0], data.shape[1], _ptr(data), _ptr(sigma), _ptr(om),
                            _ptr(psf), psf.shape[0], C.byref(o), _ptr(params), C.byref(chi2), C.byref(st))
    if rc != 0:
        raise ValueError(f"orc_fit_adam failed ({rc})")
    return params, chi2.value, st.value


def param_errors(model: Model, data, sigma, psf, params, omega=None, want_cov=False):
    data = _f32(data)
    sigma = _f32(sigma)
    psf = _f32(psf)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.uint8)
    params = _f64(params)
    err = np.empty(model.p)
    cov = np.empty((model.p, model.p)) if want_cov else None
    mc = model.c()
    lib().orc_param_errors(C.byref(mc), data.shape[0], data.shape[1], _ptr(data), _ptr(sigma), _ptr(om),
                           _ptr(psf), psf.shape[0], _ptr(params), _ptr(err), _ptr(cov))
    return (err, cov) if want_cov else err


def moments(data, sigma, omega=None, m0: float = 22.5):
    """Image moments {sky0, F0, xc, yc, m_g, r0, q0, th0 (rad), peak}."""
    data = _f32(data)
    sigma = _f32(sigma)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.uint8)
    out = np.zeros(9)
    lib().orc_moments(data.shape[0], data.shape[1], _ptr(data), _ptr(sigma), _ptr(om), float(m0), _ptr(out))
    return out


def default_guess(model: Model, data, sigma, omega=None):
    """Moment-based start vector and the 6 moment features."""
    data = _f32(data)
    sigma = _f32(sigma)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.uint8)
    params = np.zeros(model.p)
    mom = np.zeros(6)
    mc = model.c()
    rc = lib().orc_default_guess(C.byref(mc), data.shape[0], data.shape[1], _ptr(data), _ptr(sigma),
                                 _ptr(om), _ptr(params), _ptr(mom))
    if rc != 0:
        raise ValueError(f"orc_default_guess failed ({rc})")
    return params, mom


def default_guess_batch(model: Model, h, w, img_off, data, sigma, omega=None):
    """Moment-based start vectors [n][p] and moment features [n][6] of a ragged
    batch (one orc_default_guess call per galaxy)."""
    n = len(h)
    params = np.zeros((n, model.p))
    mom = np.zeros((n, 6))
    for g in range(n):
        hh, ww, o = int(h[g]), int(w[g]), int(img_off[g])
        sl = slice(o, o + hh * ww)
        om = None if omega is None else np.asarray(omega[sl]).reshape(hh, ww)
        params[g], mom[g] = default_guess(model, np.asarray(data[sl]).reshape(hh, ww),
                                          np.asarray(sigma[sl]).reshape(hh, ww), om)
    return params, mom


def fit_batch(model: Model, h, w, img_off, data, sigma, psf_k, psf_off, psf, params0, omega=None,
              max_iter=100, lambda0=1e-3, step_tol=1e-4, nthreads=None):
    """Fit a ragged batch on `nthreads` host threads (default: all cores)."""
    h = np.ascontiguousarray(h, np.int32)
    w = np.ascontiguousarray(w, np.int32)
    img_off = np.ascontiguousarray(img_off, np.int64)
    psf_k = np.ascontiguousarray(psf_k, np.int32)
    psf_off = np.ascontiguousarray(psf_off, np.int64)
    data = _f32(data)
    sigma = _f32(sigma)
    psf = _f32(psf)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.uint8)
    n = len(h)
    params = _f64(params0).reshape(n, model.p).copy()
    chi2 = np.zeros(n)
    nit = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    o = _Opts(max_iter, lambda0, step_tol)
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0))
    mc = model.c()
    lib().orc_fit_batch(C.byref(mc), n, _ptr(h), _ptr(w), _ptr(img_off), _ptr(data), _ptr(sigma), _ptr(om),
                        _ptr(psf_k), _ptr(psf_off), _ptr(psf), C.byref(o), _ptr(params), _ptr(chi2),
                        _ptr(nit), _ptr(st), int(nthreads))
    return params, chi2, nit, st


def fit_adam_batch(model: Model, h, w, img_off, data, sigma, psf_k, psf_off, psf, params0, omega=None,
                   steps=1000, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, nthreads=None):
    """Adam fits of a ragged batch on `nthreads` host threads; returns
    (params, chi2, status)."""
    h = np.ascontiguousarray(h, np.int32)
    w = np.ascontiguousarray(w, np.int32)
    img_off = np.ascontiguousarray(img_off, np.int64)
    psf_k = np.ascontiguousarray(psf_k, np.int32)
    psf_off = np.ascontiguousarray(psf_off, np.int64)
    data = _f32(data)
    sigma = _f32(sigma)
    psf = _f32(psf)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.uint8)
    n = len(h)
    params = _f64(params0).reshape(n, model.p).copy()
    chi2 = np.zeros(n)
    st = np.zeros(n, np.int32)
    o = _AdamOpts(steps, lr, beta1, beta2, eps)
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0))
    mc = model.c()
    rc = lib().orc_fit_adam_batch(C.byref(mc), n, _ptr(h), _ptr(w), _ptr(img_off), _ptr(data), _ptr(sigma),
                                  _ptr(om), _ptr(psf_k), _ptr(psf_off), _ptr(psf), C.byref(o), _ptr(params),
                                  _ptr(chi2), _ptr(st), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_fit_adam_batch failed ({rc})")
    return params, chi2, st
