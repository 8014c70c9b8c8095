"""The largest cutouts the library accepts (1024 px a side): model images and
Jacobian columns of a 1024 x 1024 and a ragged 1024 x 333 cutout (32 x 32
and 32 x 11 tiles, the last partial) against the FP64 oracle, and one LM
fit of a noisy 1024 x 1024 galaxy from the oracle's moment start (1e-4),
with the Adam fitter's per-workgroup residual image at its maximum size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import image_parity, param_parity
from tests.oracle_models import single, to_gm

PSF = S.moffat_psf(3.0, 2.0, 25)
NAMES = ["x0", "y0", "mag", "re", "n", "q", "pa", "sky"]


def _batch(shapes, data=None):
    h = np.array([s[0] for s in shapes], np.int32)
    w = np.array([s[1] for s in shapes], np.int32)
    img_off = np.concatenate([[0], np.cumsum(h.astype(np.int64) * w)[:-1]]).astype(np.int64)
    n = len(shapes)
    npix = int(img_off[-1] + h[-1] * w[-1])
    data = np.zeros(npix, np.float32) if data is None else data
    return G.Batch(h, w, img_off, np.full(n, 25, np.int32), np.arange(n, dtype=np.int64) * PSF.size, data,
                   np.ones(npix, np.float32), np.tile(PSF.ravel(), n))


def test_max_size_image_and_jacobian():
    print("max size: image and jacobian 1024x1024, 1024x333", flush=True)
    om = single(O.SERSIC, sky=True)
    gm = to_gm(om)
    shapes = [(1024, 1024), (1024, 333)]
    params = np.array([[512.3, 511.6, 12.0, 40.0, 2.5, 0.6, 30.0, 100.0],
                       [511.2, 166.7, 13.0, 25.0, 1.2, 0.4, 100.0, 50.0]])
    b = _batch(shapes)
    img = G.gm_model_image(gm, b, params).cpu().numpy()
    jac = G.gm_jacobian(gm, b, params).cpu().numpy()
    for g, (h, w) in enumerate(shapes):
        ref = O.model_image(om, h, w, PSF, params[g])
        ok, worst = image_parity(img[b.img_off[g]: b.img_off[g] + h * w].reshape(h, w), ref)
        assert ok, (g, worst)
        refj = O.jacobian(om, h, w, PSF, params[g])
        gj = jac[om.p * b.img_off[g]: om.p * (b.img_off[g] + h * w)].reshape(om.p, h, w)
        for c in range(om.p):
            err = np.max(np.abs(gj[c] - refj[c])) / np.max(np.abs(refj[c]))
            assert err <= 1e-5, (g, NAMES[c], err)


def test_max_size_fit_and_adam():
    print("max size: LM fit and Adam steps 1024x1024", flush=True)
    om = single(O.SERSIC, sky=True)
    gm = to_gm(om)
    truth = np.array([512.3, 511.6, 12.0, 40.0, 2.5, 0.6, 30.0, 100.0])
    rng = np.random.default_rng(91)
    data = (O.model_image(om, 1024, 1024, PSF, truth) + rng.normal(size=(1024, 1024))).astype(np.float32).ravel()
    b = _batch([(1024, 1024)], data=data)
    sig = np.ones_like(data)
    start, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, data, sig)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, b, start)]
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, data, sig, b.psf_k, b.psf_off, np.tile(PSF.ravel(), 1),
                                 start)
    print(f"  status gpu {gs[0]} oracle {rs[0]}; trials gpu {gn[0]} oracle {rn[0]}", flush=True)
    assert gs[0] == 0 and rs[0] == 0
    ok, worst = param_parity(NAMES, gp[0], rp[0])
    assert ok.all(), worst
    ap, ac, ast = [t.cpu().numpy() for t in G.gm_fit_adam(gm, b, start, steps=3)]
    op, oc, ost = O.fit_adam_batch(om, b.h, b.w, b.img_off, data, sig, b.psf_k, b.psf_off, np.tile(PSF.ravel(), 1),
                                   start, steps=3)
    ok, worst = param_parity(NAMES, ap[0], op[0])
    assert ok.all(), worst


def test_max_size_covariance_errors():
    """Errors sqrt(diag (J^T W J)^-1) at 1024 x 1024 and 1024 x 333 (Sec. 5.2):
    J^T W J sums a million pixels; each thread sums its FP32 partial products
    over at most 16 tiles before they enter the FP64 sums, and the errors
    (from gm_param_errors and from the fit kernel) hold the 1e-4 bar."""
    print("max size: covariance errors 1024x1024, 1024x333", flush=True)
    om = single(O.SERSIC, sky=True)
    gm = to_gm(om)
    shapes = [(1024, 1024), (1024, 333)]
    # centres inside the cutouts (x0 runs over the 333 columns): the data then
    # determine every parameter and J^T W J is well conditioned
    params = np.array([[512.3, 511.6, 12.0, 40.0, 2.5, 0.6, 30.0, 100.0],
                       [166.7, 511.2, 13.0, 25.0, 1.2, 0.4, 100.0, 50.0]])
    rng = np.random.default_rng(93)
    data = np.concatenate([(O.model_image(om, h, w, PSF, params[g]) + rng.normal(size=(h, w))).ravel()
                           for g, (h, w) in enumerate(shapes)]).astype(np.float32)
    b = _batch(shapes, data=data)
    err, cov = G.gm_param_errors(gm, b, params, want_cov=True)
    err, cov = err.cpu().numpy(), cov.cpu().numpy()
    for g, (h, w) in enumerate(shapes):
        o = int(b.img_off[g])
        re, rcov = O.param_errors(om, data[o:o + h * w].reshape(h, w), np.ones((h, w), np.float32), PSF, params[g],
                                  want_cov=True)
        rel = np.abs(err[g] - re) / re
        print(f"  {h}x{w}: worst relative error of the errors {rel.max():.2e}", flush=True)
        assert np.all(rel <= 1e-4), (g, dict(zip(NAMES, rel)))
        assert np.allclose(cov[g], rcov, rtol=1e-4, atol=1e-4 * np.sqrt(np.outer(re, re)).max())
    # errors computed by the fit kernel at its end point: equal to gm_param_errors there
    ef = torch.empty(b.n, gm.p, dtype=torch.float64, device="cuda")
    p, c, it, st = G.gm_fit_batch(gm, b, params, err_out=ef)
    ref = G.gm_param_errors(gm, b, p).cpu().numpy()
    assert np.allclose(ef.cpu().numpy(), ref, rtol=1e-5, atol=0)
