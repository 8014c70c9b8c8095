"""Pins of the oracle's free shape exponents (Sec. 4.2.2: Ferrer a and b;
Sec. 4.2.3: King alpha), beyond the finite-difference Jacobian cases of
tests/test_oracle_pins.py:

* LM recovers a, b and alpha from noise-free images rendered at known
  values, from the starts the default guess uses (a = 0.5, b = 1.9 as printed
  in Appendix C; alpha = 2);
* the Ferrer flux stays the magnitude's at free (a, b): 2-D quadrature of the
  profile (radial in the elliptical radius) against 10^(-0.4 (m - m0)).
"""
import math

import numpy as np
import pytest
import scipy.integrate as si

import oracle as O
from tests.oracle_models import single

M0 = 22.5


def _psf(k=7, s=1.2):
    c = (k - 1) / 2
    u, v = np.mgrid[0:k, 0:k]
    g = np.exp(-((u - c) ** 2 + (v - c) ** 2) / (2 * s * s))
    return (g / g.sum()).astype(np.float32)


@pytest.mark.parametrize("a,b", [(1.2, 0.8), (2.5, 1.5)])
def test_lm_recovers_ferrer_shape(orc, a, b):
    m = single(O.FERRER, sky=True, shape=True)
    H = W = 48
    psf = _psf()
    truth = np.array([24.3, 23.6, 15.0, 14.0, 0.45, 40.0, a, b, 2.0])
    d = orc.model_image(m, H, W, psf, truth).astype(np.float32)
    s = np.ones_like(d)
    start = truth.copy()
    start[[0, 1, 3, 4, 5]] += [0.3, -0.2, 1.5, 0.05, 4.0]
    start[6], start[7] = 0.5 * a + 0.4, b - 0.3
    p, chi2, nit, st = orc.fit(m, d, s, psf, start, step_tol=1e-8, max_iter=300)
    assert st == O.ST_CONVERGED, (st, nit)
    assert np.all(np.abs(p - truth) <= 1e-5 * np.maximum(np.abs(truth), 1.0)), p - truth


@pytest.mark.parametrize("alpha", [1.3, 3.5])
def test_lm_recovers_king_alpha(orc, alpha):
    m = single(O.KING, sky=True, shape=True)
    H = W = 48
    psf = _psf()
    truth = np.array([24.3, 23.6, 40.0, 2.5, 18.0, 0.8, 30.0, alpha, 1.5])
    d = orc.model_image(m, H, W, psf, truth).astype(np.float32)
    s = np.ones_like(d)
    start = truth.copy()
    start[[0, 1, 2, 3, 4]] *= [1.01, 0.99, 0.9, 1.2, 0.9]
    start[7] = 2.0
    p, chi2, nit, st = orc.fit(m, d, s, psf, start, step_tol=1e-8, max_iter=300)
    assert st == O.ST_CONVERGED, (st, nit)
    assert np.all(np.abs(p - truth) <= 1e-5 * np.maximum(np.abs(truth), 1.0)), p - truth


@pytest.mark.parametrize("a,b", [(0.5, 1.9), (1.7, -0.5), (4.0, 1.0)])
def test_ferrer_flux_at_free_shape(orc, a, b):
    m = single(O.FERRER, convolve=False, shape=True)
    F, rout, q = 12.0, 9.0, 0.6
    p = [0.0, 0.0, M0 - 2.5 * math.log10(F), rout, q, 0.0, a, b]
    # along the major axis (PA 0) the elliptical radius is |x|: integrate
    # I(r) over ellipses, area element 2 pi q r dr
    f = lambda r: 2 * math.pi * q * r * orc.profile_point(m, 0, p, r, 0.0)[0]
    got = si.quad(f, 0.0, rout, limit=400, epsabs=0, epsrel=1e-11, points=[rout * 0.999])[0]
    assert abs(got / F - 1) < 1e-8, got / F
