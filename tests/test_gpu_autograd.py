"""The adjoint (gm_model_vjp) and the torch.autograd.Function over the forward
model: against the FP64 oracle Jacobian contracted with the same pixel
weights (1e-5 of sum |J| |w| per parameter) and against central finite
differences of the FP32 forward model with h = 1e-3 relative, centres 1e-3
px (2e-3, limited by FP32 rounding of the image)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import autograd as A
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import oracle_batch
from tests.oracle_models import from_spec


def _dev(b):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf)


@pytest.mark.parametrize("cfg,n", [("sersic64", 5), ("uneven", 3), ("bulgedisk", 2)])
def test_vjp_matches_oracle_jacobian(cfg, n):
    print(f"vjp {cfg} n={n}", flush=True)
    b = oracle_batch(cfg, n, seed=11)
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    rng = np.random.default_rng(12)
    gin = rng.normal(size=b.npix).astype(np.float32)
    got = G.gm_model_vjp(gm, _dev(b), b.truth, torch.from_numpy(gin).cuda()).cpu().numpy()
    for g in range(b.n):
        h, w = int(b.h[g]), int(b.w[g])
        J = O.jacobian(om, h, w, b.psf_of(g), b.truth[g]).reshape(gm.p, -1)
        wg = b.image(gin, g).astype(np.float64).ravel()
        ref = J @ wg
        scale = np.abs(J) @ np.abs(wg)
        assert np.all(np.abs(got[g] - ref) <= 1e-5 * scale), (g, got[g], ref)


def test_autograd_function_backward_is_the_adjoint():
    b = oracle_batch("sersic64", 4, seed=13)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    db = _dev(b)
    params = torch.from_numpy(b.truth.copy()).cuda().requires_grad_(True)
    wts = torch.from_numpy(np.random.default_rng(14).normal(size=b.npix).astype(np.float32)).cuda()
    img = A.model_image(params, gm, db)
    assert torch.equal(img.detach(), G.gm_model_image(gm, db, b.truth))
    (img * wts).sum().backward()
    ref = G.gm_model_vjp(gm, db, b.truth, wts)
    assert torch.equal(params.grad, ref)


@pytest.mark.parametrize("cfg", ["sersic64", "bulgedisk"])
def test_autograd_matches_finite_differences(cfg):
    b = oracle_batch(cfg, 2, seed=15)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    db = _dev(b)
    rng = np.random.default_rng(16)
    # a smooth scalar: weighted sum of the image with positive weights
    wts = torch.from_numpy(rng.uniform(0.5, 1.5, size=b.npix).astype(np.float32)).cuda()
    # centres away from pixel edges: the oversampled window moves with floor(x0),
    # floor(y0), a step the finite differences must not straddle
    base = b.truth.copy()
    base[:, 0] = np.floor(base[:, 0]) + 0.37
    base[:, 1] = np.floor(base[:, 1]) + 0.61
    params = torch.from_numpy(base.copy()).cuda().requires_grad_(True)
    (A.model_image(params, gm, db).double() * wts.double()).sum().backward()
    grad = params.grad.cpu().numpy()
    names = S.MODEL_SPECS[b.model]["names"]
    for g in range(b.n):
        for k in range(gm.p):
            # 1e-3 relative; centres relative to the 1-px pixel scale (a step of 1e-3 x0 would
            # straddle the curvature of a cuspy high-n core)
            h = 1e-3 * (1.0 if names[k] in ("x0", "y0") else max(abs(base[g, k]), 1.0))
            vals = []
            for sgn in (1.0, -1.0):
                pp = base.copy()
                pp[g, k] += sgn * h
                img = G.gm_model_image(gm, db, pp).double()
                vals.append(float((img * wts.double()).sum().item()))
            fd = (vals[0] - vals[1]) / (2 * h)
            tol = 2e-3 * abs(grad[g, k]) + 2e-4 * np.abs(grad[g]).max()
            assert abs(fd - grad[g, k]) <= tol, (g, names[k], fd, grad[g, k])


@pytest.mark.parametrize("kind", ["sersic_box", "king_free", "ferrer_free"])
def test_vjp_new_families_match_oracle_jacobian(kind):
    """The adjoint of the boxy Sersic and of the free-shape King and Ferrer
    families, including their B, alpha and (a, b) columns."""
    from tests.gpu_helpers import oracle_box_batch, oracle_shape_batch

    print(f"vjp {kind}", flush=True)
    b = oracle_box_batch("sersic64", 3, seed=17) if kind == "sersic_box" else oracle_shape_batch("sersic64", 3, kind, 17)
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    gin = np.random.default_rng(18).normal(size=b.npix).astype(np.float32)
    got = G.gm_model_vjp(gm, _dev(b), b.truth, torch.from_numpy(gin).cuda()).cpu().numpy()
    for g in range(b.n):
        h, w = int(b.h[g]), int(b.w[g])
        J = O.jacobian(om, h, w, b.psf_of(g), b.truth[g]).reshape(gm.p, -1)
        wg = b.image(gin, g).astype(np.float64).ravel()
        ref = J @ wg
        scale = np.abs(J) @ np.abs(wg)
        assert np.all(np.abs(got[g] - ref) <= 1e-5 * scale), (g, got[g], ref)
