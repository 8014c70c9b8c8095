"""Pins of the boxy Sersic of the oracle (Sec. 4.1: the generalised radius of
eq. (r) with boxiness B and the flux factor r_box of eq. (rbox)):

* the profile integrated over the plane by 2-D quadrature (polar
  coordinates, nested adaptive quadrature of the oracle's point values) is
  the total flux 10^(-0.4 (m - m0)) for boxy and discy shapes -- this is
  what r_box is for, and a wrong r_box, exponent or axis handling fails it;
* isophotes are the generalised ellipses |X|^c + |Y/q|^c = R^c (c = B + 2)
  in the frame rotated by the position angle, and the value on them is the
  one-dimensional Sersic law at R with I_e of eq. (sersicLtot);
* r_box is 1 at B = 0 (the plain-ellipse pins of the other tests then cover
  the same code) and equals the area ratio of the unit circle and the unit
  generalised circle, the latter by direct quadrature;
* the Jacobian column of B matches finite differences (with the other
  profiles' columns in the finite-difference test).
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

import oracle as O
from tests.oracle_models import single

M0 = 22.5


def _pt(orc, m, p, x, y):
    return orc.profile_point(m, 0, p, x, y)[0]


def _total_flux(orc, m, p, re, q):
    x0, y0, th = p[0], p[1], math.radians(p[6])
    rmax = 400.0 * re / q

    def radial(phi):
        cx, sy = math.cos(phi), math.sin(phi)
        f = lambda r: r * _pt(orc, m, p, x0 + r * cx, y0 + r * sy)
        tot = 0.0
        for a, b in ((0.0, 0.3 * re), (0.3 * re, 3 * re), (3 * re, 30 * re), (30 * re, rmax)):
            tot += si.quad(f, a, b, limit=200, epsabs=0, epsrel=1e-10)[0]
        return tot

    kinks = sorted(((th + k * math.pi / 2) % (2 * math.pi)) for k in range(4))
    edges = [0.0] + kinks + [2 * math.pi]
    return sum(si.quad(radial, a, b, limit=200, epsabs=0, epsrel=1e-9)[0] for a, b in zip(edges, edges[1:])
               if b > a)


@pytest.mark.parametrize("B,n", [(0.0, 1.0), (0.8, 1.0), (-0.5, 2.5), (1.5, 0.8)])
def test_boxy_total_flux_is_the_magnitude(orc, B, n):
    m = single(O.SERSIC, convolve=False, box=True)
    F = 37.0
    re, q = 3.0, 0.7
    p = [0.0, 0.0, M0 - 2.5 * math.log10(F), re, n, q, 30.0, B]
    got = _total_flux(orc, m, p, re, q)
    assert abs(got / F - 1) < 2e-6, got / F


@pytest.mark.parametrize("B", [-0.6, 0.7, 1.8])
def test_boxy_isophotes_are_generalised_ellipses(orc, B):
    m = single(O.SERSIC, convolve=False, box=True)
    c = B + 2.0
    n, re, q, pa, F = 1.7, 4.0, 0.6, 25.0, 50.0
    p = [3.0, -2.0, M0 - 2.5 * math.log10(F), re, n, q, pa, B]
    th = math.radians(pa)
    b = sp.gammaincinv(2 * n, 0.5)
    rbox = math.pi * c / (2 * sp.beta(1 / c, 1 / c))
    Ie = rbox * F * b ** (2 * n) / (2 * math.pi * q * re * re * n * sp.gamma(2 * n) * math.exp(b))
    for R in (0.7, 4.0, 9.0):
        want = Ie * math.exp(-b * ((R / re) ** (1 / n) - 1))
        for phi in np.linspace(0.05, 2 * math.pi, 17):
            u, v = math.cos(phi), math.sin(phi)
            s = R / (abs(u) ** c + abs(v / q) ** c) ** (1 / c)
            X, Y = s * u, s * v
            x = p[0] + math.cos(th) * X - math.sin(th) * Y
            y = p[1] + math.sin(th) * X + math.cos(th) * Y
            assert abs(_pt(orc, m, p, x, y) / want - 1) < 1e-11, (R, phi)


def test_rbox_is_the_area_ratio(orc):
    # I_e scales by r_box = (area of the unit circle) / (area of |x|^c + |y|^c <= 1);
    # compare the central intensities at B and at 0 with that ratio, the area by quadrature
    m = single(O.SERSIC, convolve=False, box=True)
    for B in (-0.7, 0.0, 0.9, 2.0):
        c = B + 2.0
        area = 4 * si.quad(lambda x: (1 - x ** c) ** (1 / c), 0, 1, epsabs=0, epsrel=1e-12)[0]
        p = [0.0, 0.0, 20.0, 3.0, 1.0, 0.8, 10.0, B]
        p0 = list(p[:7]) + [0.0]
        ratio = _pt(orc, m, p, 0.0, 0.0) / _pt(orc, m, p0, 0.0, 0.0)
        assert abs(ratio / (math.pi / area) - 1) < 1e-10, (B, ratio)


def _psf(k=7, s=1.2):
    cc = (k - 1) / 2
    u, v = np.mgrid[0:k, 0:k]
    g = np.exp(-((u - cc) ** 2 + (v - cc) ** 2) / (2 * s * s))
    return (g / g.sum()).astype(np.float32)


@pytest.mark.parametrize("B", [0.6, -0.35])
def test_lm_recovers_boxiness_from_noise_free_data(orc, B):
    m = single(O.SERSIC, sky=True, box=True)
    H = W = 40
    psf = _psf()
    truth = np.array([20.3, 19.6, 16.0, 4.0, 2.2, 0.65, 40.0, B, 3.0])
    d = orc.model_image(m, H, W, psf, truth).astype(np.float32)
    s = np.ones_like(d)
    start = truth * np.array([1, 1, 1, 1.2, 0.8, 1.1, 1, 0, 0.8]) + np.array([0.4, -0.3, 0.2, 0, 0, 0, 6, 0, 0])
    p, chi2, nit, st = orc.fit(m, d, s, psf, start, step_tol=1e-8)
    assert st == O.ST_CONVERGED
    assert np.all(np.abs(p - truth) <= 1e-5 * np.maximum(np.abs(truth), 1.0)), p - truth
