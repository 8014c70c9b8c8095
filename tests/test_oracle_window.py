"""Pin of the oracle's oversampled central window.

The rule (the paper has no sub-pixel sampling; this build's reading): for
every radial component, the pixels of rows floor(H - y0) - h .. + h and columns
floor(x0) - h .. + h (h = os_window // 2, clipped to the cutout) take the mean
of the profile over the f x f sub-pixel centres (j + (s + 1/2)/f,
H - i - (t + 1/2)/f); every other pixel takes the profile at its centre
(j + 1/2, H - i - 1/2), the grid of Appendix C with y growing upwards.

The profile here is a circular Sersic of index 1/2, which is a Gaussian
(Sec. 4.1 with nu_{1/2} = ln 2): I = F / (2 pi s^2) exp(-r^2 / (2 s^2)) with
s^2 = r_e^2 / (2 ln 2).  Its pixel integral is a product of two erf
differences, so each window pixel is checked three ways, none of them through
the oracle's own code: against the closed form sampled at the 10 x 10
sub-pixel centres (to rounding), against the exact erf integral within the
error bound of the composite midpoint rule, and as different from the centre
sample; every pixel outside the window equals the closed form at its centre.
A row convention of floor(y0) for floor(H - y0), a half-width off by one, or
sub-samples shifted by half a sub-pixel each fail one of these.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.oracle_models import single

F = 50.0
M0 = 22.5


def _gauss_sigma(re):
    return re / math.sqrt(2.0 * math.log(2.0))


def _closed_form(x, y, x0, y0, re):
    s = _gauss_sigma(re)
    return F / (2 * math.pi * s * s) * np.exp(-((x - x0) ** 2 + (y - y0) ** 2) / (2 * s * s))


def _closed_dx0(x, y, x0, y0, re):
    s = _gauss_sigma(re)
    return _closed_form(x, y, x0, y0, re) * (x - x0) / (s * s)


def _closed_dy0(x, y, x0, y0, re):
    s = _gauss_sigma(re)
    return _closed_form(x, y, x0, y0, re) * (y - y0) / (s * s)


def _rel_tol(x, y, x0, y0, re):
    # exp(-a) carries a relative rounding of a few a ulp (nu_n and ln I_e are
    # computed, not exact, on the oracle side)
    s = _gauss_sigma(re)
    return 2e-15 * (16.0 + ((x - x0) ** 2 + (y - y0) ** 2) / (2 * s * s))


def _erf_pixel_mean(i, j, H, x0, y0, re):
    """Exact mean of the Gaussian over pixel (i, j): x in [j, j+1], y in [H-i-1, H-i]."""
    s = _gauss_sigma(re)
    k = 1.0 / (math.sqrt(2.0) * s)
    ix = 0.5 * (math.erf((j + 1 - x0) * k) - math.erf((j - x0) * k))
    iy = 0.5 * (math.erf((H - i - y0) * k) - math.erf((H - i - 1 - y0) * k))
    return F * ix * iy


def _midpoint_bound(re, f):
    """|mean of f x f midpoint samples - exact mean| for one pixel.

    Per axis the Gaussian factor g (peak 1/(sqrt(2 pi) s) times the unit
    interval) has |g''| <= g(0)/s^2, so the composite midpoint rule with step
    1/f errs by at most e = g(0)/(24 f^2 s^2); the product of the two axes'
    means then errs by at most 2 e G + e^2 with G = g(0) >= each factor.
    """
    s = _gauss_sigma(re)
    g0 = 1.0 / (math.sqrt(2 * math.pi) * s)
    e = g0 / (24.0 * f * f * s * s)
    return F * (2 * e * g0 + e * e)


def _window(H, W, x0, y0, osw):
    h = osw // 2
    ic, jc = math.floor(H - y0), math.floor(x0)
    return (max(ic - h, 0), min(ic + h, H - 1), max(jc - h, 0), min(jc + h, W - 1))


CASES = [
    # H, W, x0, y0, r_e, os_window
    (16, 16, 8.0, 8.0, 1.2, 5),                # centre on a pixel corner
    (16, 16, 7.999999, 8.000001, 1.2, 5),      # just across that corner
    (13, 20, 6.3, 3.3, 1.5, 5),                # H != W: floor(H - y0) = 9, floor(y0) = 3
    (13, 20, 12.71, 9.42, 0.9, 5),
    (12, 12, 0.3, 11.7, 1.1, 5),               # window clipped at the top-left corner
    (12, 12, 11.99, 0.01, 1.3, 5),             # ... at the bottom-right corner
    (9, 11, 5.5, 4.5, 1.0, 3),                 # a 3 x 3 window
    (9, 11, 2.25, 6.75, 1.4, 7),               # a 7 x 7 window
]


@pytest.mark.parametrize("H,W,x0,y0,re,osw", CASES)
def test_oversampling_window_rule(orc, H, W, x0, y0, re, osw):
    f = 10
    m = single(O.SERSIC, convolve=False, oversample=f)
    m.os_window = osw
    params = [x0, y0, M0 - 2.5 * math.log10(F), re, 0.5, 1.0, 0.0]
    img = orc.model_image(m, H, W, np.ones((1, 1), np.float32), params)
    jac = orc.jacobian(m, H, W, np.ones((1, 1), np.float32), params)
    i0, i1, j0, j1 = _window(H, W, x0, y0, osw)
    sub = (np.arange(f) + 0.5) / f
    bound = _midpoint_bound(re, f)
    n_in = 0
    for i in range(H):
        for j in range(W):
            xc, yc = j + 0.5, H - i - 0.5
            centre = _closed_form(xc, yc, x0, y0, re)
            if i0 <= i <= i1 and j0 <= j <= j1:
                n_in += 1
                xs, ys = np.meshgrid(j + sub, H - i - sub)
                mid = _closed_form(xs, ys, x0, y0, re).mean()
                # the 10 x 10 sub-pixel centres, to rounding
                assert abs(img[i, j] - mid) <= 1e-12 * mid + 1e-300, (i, j)
                # an integral of the pixel: within the midpoint rule's bound of erf
                exact = _erf_pixel_mean(i, j, H, x0, y0, re)
                assert abs(img[i, j] - exact) <= bound, (i, j, img[i, j], exact, bound)
                # and not the centre sample
                assert abs(img[i, j] - centre) > 1e-9 * centre, (i, j)
                # derivatives follow the same rule
                for col, fn in ((0, _closed_dx0), (1, _closed_dy0)):
                    dmid = fn(xs, ys, x0, y0, re).mean()
                    scale = np.abs(fn(xs, ys, x0, y0, re)).max()
                    assert abs(jac[col, i, j] - dmid) <= 1e-11 * scale + 1e-300, (col, i, j)
            else:
                tol = _rel_tol(xc, yc, x0, y0, re)
                assert abs(img[i, j] - centre) <= tol * centre + 1e-300, (i, j)
                for col, fn in ((0, _closed_dx0), (1, _closed_dy0)):
                    dv = fn(xc, yc, x0, y0, re)
                    assert abs(jac[col, i, j] - dv) <= 4 * tol * abs(dv) + 1e-300, (col, i, j)
    assert n_in == (i1 - i0 + 1) * (j1 - j0 + 1) > 0


def test_window_sits_on_the_pixel_holding_the_centre(orc):
    # The pixel whose value deviates most from its centre sample is the one that
    # holds (x0, y0): at a cusp-free Gaussian the curvature is largest there.
    H, W, x0, y0, re = 13, 20, 6.3, 3.3, 1.5
    m = single(O.SERSIC, convolve=False, oversample=10)
    params = [x0, y0, M0 - 2.5 * math.log10(F), re, 0.5, 1.0, 0.0]
    img = orc.model_image(m, H, W, np.ones((1, 1), np.float32), params)
    m1 = single(O.SERSIC, convolve=False, oversample=1)
    pt = orc.model_image(m1, H, W, np.ones((1, 1), np.float32), params)
    dev = np.abs(img - pt)
    i, j = np.unravel_index(np.argmax(dev), dev.shape)
    assert (i, j) == (H - 1 - int(y0), int(x0)) == (9, 6)
    # exactly 25 pixels differ from point sampling
    assert int((dev > 0).sum()) == 25


def test_oversampling_off_is_point_sampling(orc):
    H, W, x0, y0, re = 10, 10, 4.7, 5.2, 1.1
    m = single(O.SERSIC, convolve=False, oversample=1)
    params = [x0, y0, M0 - 2.5 * math.log10(F), re, 0.5, 1.0, 0.0]
    img = orc.model_image(m, H, W, np.ones((1, 1), np.float32), params)
    jj, ii = np.meshgrid(np.arange(W), np.arange(H))
    ref = _closed_form(jj + 0.5, H - ii - 0.5, x0, y0, re)
    assert np.all(np.abs(img - ref) <= _rel_tol(jj + 0.5, H - ii - 0.5, x0, y0, re) * ref + 1e-300)
