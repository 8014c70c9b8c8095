"""Pins of the oracle's gradient-descent fitter (Adam on chi^2, the paper's
own fitter of Sec. 5.1) against what fixes it independently of its code:

* a plain re-derivation of Adam's update (Kingma and Ba 2015, Algorithm 1)
  driven by central finite differences of chi^2, where chi^2 comes from the
  oracle's forward model image (pinned elsewhere) and the definition of
  Sec. 5.1; it would catch a wrong sign, a dropped bias correction, a wrong
  factor in the gradient or a swapped moment;
* the special case beta1 = beta2 = 0, where Adam is sign descent: every free
  variable moves by exactly lr per step, against the sign of the gradient;
* the minimum: with a small rate Adam ends at the chi^2 minimum that the LM
  finds (the two minimise the same chi^2);
* zero steps: the start, canonicalised, and chi^2 at it from its definition.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.oracle_models import single


def _psf(k=7, s=1.2):
    c = (k - 1) / 2
    u, v = np.mgrid[0:k, 0:k]
    g = np.exp(-((u - c) ** 2 + (v - c) ** 2) / (2 * s * s))
    return (g / g.sum()).astype(np.float32)


# Sersic + sky columns: x0 y0 mag re n q pa sky.  The fit variables are the
# natural values except ln re, ln n and PA in radians.
LOGS = (3, 4)
PA = 6


def _to_u(p):
    u = np.array(p, float)
    u[list(LOGS)] = np.log(u[list(LOGS)])
    u[PA] = math.radians(u[PA])
    return u


def _from_u(u):
    p = np.array(u, float)
    p[list(LOGS)] = np.exp(p[list(LOGS)])
    p[PA] = math.degrees(p[PA])
    return p


def _problem(orc, seed=0, H=20, W=22):
    m = single(O.SERSIC, sky=True)
    psf = _psf()
    truth = np.array([10.3, 9.6, 16.5, 3.2, 1.6, 0.6, 40.0, 2.0])
    rng = np.random.default_rng(seed)
    sig = rng.uniform(0.8, 1.5, (H, W)).astype(np.float32)
    d = (orc.model_image(m, H, W, psf, truth) + sig * rng.normal(size=(H, W))).astype(np.float32)
    start = np.array([10.45, 9.5, 16.8, 3.8, 1.3, 0.52, 35.0, 1.5])
    return m, psf, d, sig, truth, start


def _chi2(orc, m, psf, d, sig, p):
    """chi^2 of Sec. 5.1 from the model image: sum over pixels of ((D - M) / sigma)^2."""
    mod = orc.model_image(m, d.shape[0], d.shape[1], psf, p)
    r = (d.astype(np.float64) - mod) / sig.astype(np.float64)
    return float(np.sum(r * r))


def _fd_grad(orc, m, psf, d, sig, u, h=1e-5):
    g = np.zeros(len(u))
    for k in range(len(u)):
        up, um = u.copy(), u.copy()
        up[k] += h
        um[k] -= h
        g[k] = (_chi2(orc, m, psf, d, sig, _from_u(up)) - _chi2(orc, m, psf, d, sig, _from_u(um))) / (2 * h)
    return g


def _adam_reference(orc, m, psf, d, sig, p0, steps, lr, b1, b2, eps):
    u = _to_u(p0)
    mt = np.zeros(len(u))
    vt = np.zeros(len(u))
    for t in range(1, steps + 1):
        g = _fd_grad(orc, m, psf, d, sig, u)
        mt = b1 * mt + (1 - b1) * g
        vt = b2 * vt + (1 - b2) * g * g
        u = u - lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
    return u


@pytest.mark.parametrize("b1,b2", [(0.9, 0.999), (0.6, 0.8)])
def test_adam_steps_match_finite_difference_adam(orc, b1, b2):
    m, psf, d, sig, _, start = _problem(orc)
    steps, lr, eps = 4, 0.02, 1e-8
    ref_u = _adam_reference(orc, m, psf, d, sig, start, steps, lr, b1, b2, eps)
    p, chi2, st = orc.fit_adam(m, d, sig, psf, start, steps=steps, lr=lr, beta1=b1, beta2=b2, eps=eps)
    assert st == O.ST_MAXITER
    got_u = _to_u(p)
    assert np.all(np.abs(got_u - ref_u) < 1e-7), got_u - ref_u
    assert abs(chi2 / _chi2(orc, m, psf, d, sig, p) - 1) < 1e-10


def test_adam_without_moments_is_sign_descent(orc):
    m, psf, d, sig, _, start = _problem(orc, seed=1)
    lr = 0.01
    g = _fd_grad(orc, m, psf, d, sig, _to_u(start))
    p, _, _ = orc.fit_adam(m, d, sig, psf, start, steps=1, lr=lr, beta1=0.0, beta2=0.0, eps=1e-12)
    du = _to_u(p) - _to_u(start)
    assert np.allclose(du, -lr * np.sign(g), rtol=0, atol=1e-12), (du, g)


def test_adam_reaches_the_lm_minimum(orc):
    m, psf, d, sig, truth, start = _problem(orc, seed=2)
    lp, lchi2, _, lst = orc.fit(m, d, sig, psf, start, step_tol=1e-8)
    assert lst == O.ST_CONVERGED
    ap, achi2, ast = orc.fit_adam(m, d, sig, psf, start, steps=3000, lr=0.01)
    assert ast == O.ST_MAXITER
    # the LM point is the minimum; Adam ends within a hair of it
    assert lchi2 <= achi2 * (1 + 1e-12)
    assert achi2 - lchi2 < 1e-6 * lchi2
    err = orc.param_errors(m, d, sig, psf, lp)
    assert np.all(np.abs(ap - lp) < 0.01 * err), (ap - lp) / err


def test_adam_zero_steps_returns_the_canonical_start(orc):
    m, psf, d, sig, _, _ = _problem(orc, seed=3)
    start = np.array([10.2, 9.7, 16.6, 2.5, 1.5, 1.6, 100.0, 1.8])     # q > 1
    p, chi2, st = orc.fit_adam(m, d, sig, psf, start, steps=0)
    canon = orc.canonicalise(m, start)
    assert st == O.ST_MAXITER
    assert np.allclose(p, canon, rtol=1e-14, atol=1e-12)
    assert abs(canon[5] - 1 / 1.6) < 1e-14 and abs(canon[3] - 2.5 * 1.6) < 1e-12
    assert abs(chi2 / _chi2(orc, m, psf, d, sig, start) - 1) < 1e-12
