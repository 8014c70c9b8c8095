"""The paper-shaped workload (128x128 cutouts, 41x41 Moffat PSF: the
compile-time PSF side 41 of the Sersic kernels) against the FP64 oracle:
model images (1e-5), Jacobian columns (1e-5) and fits from each side's own
moment start (1e-4)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import image_parity, oracle_batch, param_parity
from tests.oracle_models import from_spec


@pytest.fixture(scope="module")
def paper():
    print("building paper-shaped galaxies 0..5 (seed 0)", flush=True)
    return oracle_batch("paper", 6, seed=0)


def _dev(b):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf)


def test_paper_model_image_and_jacobian(paper):
    b = paper.subset(range(3))
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    img = G.gm_model_image(gm, _dev(b), b.truth).cpu().numpy()
    jac = G.gm_jacobian(gm, _dev(b), b.truth).cpu().numpy()
    for g in range(b.n):
        ref = O.model_image(om, 128, 128, b.psf_of(g), b.truth[g])
        ok, worst = image_parity(b.image(img, g), ref)
        assert ok, (g, worst)
        refj = O.jacobian(om, 128, 128, b.psf_of(g), b.truth[g])
        gj = jac[gm.p * b.img_off[g]: gm.p * (b.img_off[g] + 128 * 128)].reshape(gm.p, 128, 128)
        for c in range(gm.p):
            err = np.max(np.abs(gj[c] - refj[c])) / np.max(np.abs(refj[c]))
            assert err <= 1e-5, (g, c, err)


def test_paper_fits(paper):
    b = paper
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    db = _dev(b)
    start, _ = G.gm_default_guess(gm, db)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start)]
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, ostart)
    names = S.MODEL_SPECS[b.model]["names"]
    both = (gs == 0) & (rs == 0)
    npass = sum(int(param_parity(names, gp[g], rp[g], sky_sigma=float(np.median(b.image(b.sigma, g))))[0].all())
                for g in np.where(both)[0])
    print(f"paper-shaped fits: {npass}/{int(both.sum())} within 1e-4; iterations gpu {gn.mean():.1f} "
          f"oracle {rn.mean():.1f}", flush=True)
    assert both.sum() >= 0.8 * b.n and npass == both.sum()
