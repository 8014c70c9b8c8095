"""A batch whose galaxies have different PSF sides (5, 15, 25, 31): the
library then runs its generic-side kernels (taps read from LDS one by one,
region geometry per galaxy, LDS sized for the largest side).  Model images,
LM fits from the oracle's moment start and 12 Adam steps against the FP64
oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import image_parity, param_parity
from tests.oracle_models import from_spec

SIDES = [5, 15, 25, 31]


def _batch():
    b = S.draw("uneven", len(SIDES), seed=93)
    psfs = [S.moffat_psf(3.0, 2.0, k) for k in SIDES]
    b.psf_k = np.array(SIDES, np.int32)
    b.psf_off = np.concatenate([[0], np.cumsum([k * k for k in SIDES])[:-1]]).astype(np.int64)
    b.psf = np.concatenate([p.ravel() for p in psfs]).astype(np.float32)
    m = from_spec(b.model)
    ut = S.unit_truth(b)
    units = np.concatenate([O.model_image(m, int(b.h[g]), int(b.w[g]), b.psf_of(g), ut[g]).ravel()
                            for g in range(b.n)])
    return S.finish(b, units)


def test_mixed_psf_sides_images_fits_and_adam():
    print(f"mixed PSF sides {SIDES}", flush=True)
    b = _batch()
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    names = S.MODEL_SPECS[b.model]["names"]
    db = G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf)
    img = G.gm_model_image(gm, db, b.truth).cpu().numpy()
    for g in range(b.n):
        ref = O.model_image(om, int(b.h[g]), int(b.w[g]), b.psf_of(g), b.truth[g])
        ok, worst = image_parity(b.image(img, g), ref)
        assert ok, (g, SIDES[g], worst)
    start, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start)]
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, start)
    print(f"  LM status gpu {gs.tolist()} oracle {rs.tolist()}", flush=True)
    for g in np.where((gs == 0) & (rs == 0))[0]:
        ok, worst = param_parity(names, gp[g], rp[g], sky_sigma=float(np.median(b.image(b.sigma, g))))
        assert ok.all(), (g, SIDES[g], worst)
    assert ((gs == 0) & (rs == 0)).sum() >= len(SIDES) - 1
    ap, ac, ast = [t.cpu().numpy() for t in G.gm_fit_adam(gm, db, start, steps=12)]
    op, oc, ost = O.fit_adam_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, start,
                                   steps=12)
    for g in range(b.n):
        ok, worst = param_parity(names, ap[g], op[g], sky_sigma=float(np.median(b.image(b.sigma, g))))
        assert ok.all(), (g, SIDES[g], worst)
