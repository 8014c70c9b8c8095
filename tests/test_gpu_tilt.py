"""Single Sersic + the tilted-plane sky (Appendix D, eq. new_sky_I) on the
HIP path against the FP64 oracle: model images (1e-5), Jacobian columns
(1e-5; the sky's columns are analytic), start vectors (1e-6), covariance
errors (1e-4) and fits from each side's own moment start (1e-4).  The data
are oracle-rendered galaxies plus a sky plane added on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import image_parity, oracle_batch, param_parity
from tests.oracle_models import from_spec

NAMES = S.MODEL_SPECS["sersic_tilt"]["names"]


def _tilted(cfg, n, seed):
    """Galaxies of `cfg` with a sky plane: truth [.., sky, kx, ky]."""
    b = oracle_batch(cfg, n, seed=seed)
    rng = np.random.default_rng(seed + 100)
    truth = np.zeros((b.n, 10))
    truth[:, :8] = b.truth
    noise = np.median(b.sigma)
    for g in range(b.n):
        h, w = int(b.h[g]), int(b.w[g])
        kx, ky = rng.uniform(-0.02, 0.02, 2) * noise
        x = np.arange(w) + 0.5 - w / 2
        y = h - np.arange(h) - 0.5 - h / 2
        o = int(b.img_off[g])
        b.data[o:o + h * w] += (kx * x[None, :] + ky * y[:, None]).astype(np.float32).ravel()
        truth[g, 8:] = kx, ky
    return b, truth


def _dev(b):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf)


@pytest.mark.parametrize("cfg", ["sersic64", "uneven"])
def test_tilt_model_image_and_jacobian(cfg):
    b, truth = _tilted(cfg, 3, seed=61)
    om = from_spec("sersic_tilt")
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic_tilt"])
    truth[:, 8:] = [[0.3, -0.2], [-0.1, 0.4], [0.05, 0.05]]      # visible planes
    img = G.gm_model_image(gm, _dev(b), truth).cpu().numpy()
    jac = G.gm_jacobian(gm, _dev(b), truth).cpu().numpy()
    for g in range(b.n):
        h, w = int(b.h[g]), int(b.w[g])
        ref = O.model_image(om, h, w, b.psf_of(g), truth[g])
        ok, worst = image_parity(b.image(img, g), ref)
        assert ok, (g, worst)
        refj = O.jacobian(om, h, w, b.psf_of(g), truth[g])
        gj = jac[10 * b.img_off[g]: 10 * (b.img_off[g] + h * w)].reshape(10, h, w)
        for c in range(10):
            err = np.max(np.abs(gj[c] - refj[c])) / np.max(np.abs(refj[c]))
            assert err <= 1e-5, (g, NAMES[c], err)


def test_tilt_guess_errors_and_fits():
    b, truth = _tilted("sersic64", 24, seed=62)
    om = from_spec("sersic_tilt")
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic_tilt"])
    db = _dev(b)
    start, mom = G.gm_default_guess(gm, db)
    start = start.cpu().numpy()
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    assert np.allclose(start, ostart, rtol=1e-6, atol=1e-9)
    err = G.gm_param_errors(gm, db, truth).cpu().numpy()
    for g in range(4):
        re = O.param_errors(om, b.image(b.data, g), b.image(b.sigma, g), b.psf_of(g), truth[g])
        assert np.allclose(err[g], re, rtol=1e-4, atol=0), (g, err[g], re)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start)]
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, ostart)
    both = (gs == 0) & (rs == 0)
    npass = 0
    for g in np.where(both)[0]:
        ok, worst = param_parity(NAMES, gp[g], rp[g], sky_sigma=float(np.median(b.image(b.sigma, g))))
        npass += int(ok.all())
    print(f"tilted sky fits: {npass}/{int(both.sum())} within 1e-4 of {b.n}; iterations gpu {gn.mean():.1f} "
          f"oracle {rn.mean():.1f}; kx, ky recovered within 3 sigma: "
          f"{np.mean(np.abs(gp[both, 8:] - truth[both, 8:]) < 3 * err[both, 8:]):.2f}", flush=True)
    assert both.sum() >= 0.8 * b.n and npass == both.sum()
