"""Free shape exponents on the HIP path against the FP64 oracle: Ferrer a, b
(Sec. 4.2.2) and King alpha (Sec. 4.2.3) as LM variables.  Model images
(1e-5), Jacobian columns (1e-5) at PSF sides 15 and 25, start vectors (1e-6)
and fits of oracle-rendered noisy galaxies from the oracle's moment start
(1e-4)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import image_parity, judge_fit
from tests.oracle_models import single, to_gm

NAMES = {O.FERRER: ["x0", "y0", "mag", "rout", "q", "pa", "a", "b", "sky"],
         O.KING: ["x0", "y0", "I0", "rc", "rt", "q", "pa", "alpha", "sky"]}
# a smooth Ferrer (a >= 1) so that the derivative planes hold 1e-5 at r_out
CASES = {
    O.FERRER: [[40.3, 37.6, 12.5, 16.0, 0.55, 40.0, 1.6, 0.7, 2.0], [38.1, 41.2, 12.0, 12.0, 0.7, 120.0, 2.8, 1.2, 1.0]],
    O.KING: [[40.3, 37.6, 300.0, 2.5, 25.0, 0.8, 60.0, 2.7, 2.0], [38.1, 41.2, 200.0, 3.5, 30.0, 0.9, 10.0, 1.4, 1.0]],
}


def _batch(shapes, psf, data=None, sigma=None):
    h = np.array([s[0] for s in shapes], np.int32)
    w = np.array([s[1] for s in shapes], np.int32)
    img_off = np.concatenate([[0], np.cumsum(h.astype(np.int64) * w)[:-1]]).astype(np.int64)
    n = len(shapes)
    k = np.full(n, psf.shape[0], np.int32)
    psf_off = np.arange(n, dtype=np.int64) * psf.size
    npix = int(img_off[-1] + h[-1] * w[-1])
    data = np.zeros(npix, np.float32) if data is None else data
    sigma = np.ones(npix, np.float32) if sigma is None else sigma
    return G.Batch(h, w, img_off, k, psf_off, data, sigma, np.tile(psf.ravel(), n))


@pytest.mark.parametrize("typ", [O.FERRER, O.KING])
@pytest.mark.parametrize("k", [15, 25])
def test_free_shape_image_and_jacobian(typ, k):
    print(f"free shape image/jacobian type {typ} K={k}", flush=True)
    om = single(typ, sky=True, shape=True)
    gm = to_gm(om)
    psf = S.moffat_psf(3.0, 2.0, k)
    shapes = [(80, 76), (71, 90)]
    params = np.array(CASES[typ])
    b = _batch(shapes, psf)
    img = G.gm_model_image(gm, b, params).cpu().numpy()
    jac = G.gm_jacobian(gm, b, params).cpu().numpy()
    for g, (h, w) in enumerate(shapes):
        ref = O.model_image(om, h, w, psf, params[g])
        ok, worst = image_parity(img[b.img_off[g]: b.img_off[g] + h * w].reshape(h, w), ref)
        assert ok, (g, worst)
        refj = O.jacobian(om, h, w, psf, params[g])
        gj = jac[om.p * b.img_off[g]: om.p * (b.img_off[g] + h * w)].reshape(om.p, h, w)
        for c in range(om.p):
            err = np.max(np.abs(gj[c] - refj[c])) / np.max(np.abs(refj[c]))
            assert err <= 1e-5, (g, NAMES[typ][c], err)


@pytest.mark.parametrize("typ", [O.FERRER, O.KING])
def test_free_shape_fits(typ):
    om = single(typ, sky=True, shape=True)
    gm = to_gm(om)
    psf = S.moffat_psf(3.0, 2.0, 15)
    rng = np.random.default_rng(81 + typ)
    n, H, W = 16, 80, 80
    truth = np.array(CASES[typ][0] * n, float).reshape(n, -1)
    truth[:, 0] += rng.uniform(-2, 2, n)
    truth[:, 1] += rng.uniform(-2, 2, n)
    truth[:, NAMES[typ].index("pa")] = rng.uniform(0, 180, n)
    if typ == O.FERRER:
        truth[:, 6] = rng.uniform(1.0, 3.0, n)
        truth[:, 7] = rng.uniform(0.0, 1.5, n)
    else:
        truth[:, 7] = rng.uniform(1.2, 4.0, n)
    data = np.concatenate([(O.model_image(om, H, W, psf, truth[g]) + rng.normal(size=(H, W))).ravel()
                           for g in range(n)]).astype(np.float32)
    b = _batch([(H, W)] * n, psf, data=data)
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, data, b.sigma.cpu().numpy())
    gstart, _ = G.gm_default_guess(gm, b)
    assert np.allclose(gstart.cpu().numpy(), ostart, rtol=1e-6, atol=1e-9)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, b, ostart)]
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, data, b.sigma.cpu().numpy(), b.psf_k, b.psf_off,
                                 b.psf.cpu().numpy(), ostart)
    both = (gs == 0) & (rs == 0)
    npass, fails, counts = 0, [], {}
    sig = b.sigma.cpu().numpy()
    for g in np.where(both)[0]:
        o = int(b.img_off[g])
        ok, how, worst = judge_fit(om, NAMES[typ], data[o:o + H * W].reshape(H, W), sig[o:o + H * W].reshape(H, W),
                                   psf, gp[g], rp[g], gc[g], rc[g])
        counts[how] = counts.get(how, 0) + 1
        npass += bool(ok)
        if not ok:
            fails.append((int(g), round(worst, 2)))
    print(f"free shape fits type {typ}: {npass}/{int(both.sum())} pass {counts}; converged gpu {np.mean(gs == 0):.2f} "
          f"oracle {np.mean(rs == 0):.2f}; fails {fails[:4]}", flush=True)
    assert np.mean(rs == 0) >= 0.6
    assert npass == both.sum()


@pytest.mark.parametrize("typ", [O.FERRER, O.KING])
def test_free_shape_covariance_errors(typ):
    om = single(typ, sky=True, shape=True)
    gm = to_gm(om)
    psf = S.moffat_psf(3.0, 2.0, 15)
    params = np.array(CASES[typ])
    rng = np.random.default_rng(85 + typ)
    data = np.concatenate([(O.model_image(om, 80, 80, psf, params[g]) + rng.normal(size=(80, 80))).ravel()
                           for g in range(2)]).astype(np.float32)
    b = _batch([(80, 80)] * 2, psf, data=data)
    err = G.gm_param_errors(gm, b, params).cpu().numpy()
    for g in range(2):
        ref = O.param_errors(om, data[g * 6400:(g + 1) * 6400].reshape(80, 80), np.ones((80, 80), np.float32), psf,
                             params[g])
        assert np.allclose(err[g], ref, rtol=1e-4, atol=0), (g, err[g], ref)
