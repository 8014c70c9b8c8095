"""Faulty inputs on the HIP path against the FP64 oracle.

Pixels: a NaN or infinite data value, and a sigma that is zero, negative, NaN
or infinite, give the pixel weight 0 (w = Omega / sigma^2 of Sec. 5.1 with
such pixels masked) in the moments, the start vector, chi^2, the normal
equations and the covariance errors, on both sides.

Start vectors: a NaN in any column gives a non-finite chi^2 at the start and
status NONFINITE without a trial (the bounds never turn a NaN into a finite
value); an infinite centre, scale or index is clamped to its bound (the fit starts
there);
a magnitude of -inf (infinite flux) or an infinite position angle leaves
chi^2 non-finite (NONFINITE); a
boxiness outside its bounds is clamped before the first evaluation.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import judge_batch, oracle_batch, oracle_box_batch
from tests.oracle_models import from_spec


def _dev(b):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf, omega=b.omega)


def _plant_faults(b, seed):
    """Scatter faulty pixels over each cutout: at the centre, in the border
    frame the sky estimate uses, and at random places."""
    rng = np.random.default_rng(seed)
    bad_d = [np.nan, np.inf, -np.inf]
    bad_s = [0.0, -1.0, np.nan, np.inf, -np.inf]
    for g in range(b.n):
        h, w, o = int(b.h[g]), int(b.w[g]), int(b.img_off[g])
        cells = [(h // 2, w // 2), (h // 2 + 1, w // 2 - 1), (0, 0), (1, w - 1), (h - 1, 3)]
        cells += [tuple(rng.integers(0, [h, w])) for _ in range(40)]
        for c, (i, j) in enumerate(cells):
            ix = o + int(i) * w + int(j)
            if c % 2 == 0:
                b.data[ix] = bad_d[c % len(bad_d)]
            else:
                b.sigma[ix] = bad_s[c % len(bad_s)]
    return b


def test_faulty_pixels_are_weightless():
    b = _plant_faults(oracle_batch("sersic64", 16, seed=61), 61)
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    names = S.MODEL_SPECS[b.model]["names"]
    db = _dev(b)
    # start vectors and moments
    gstart, gmom = [t.cpu().numpy() for t in G.gm_default_guess(gm, db)]
    ostart, omom = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    assert np.all(np.isfinite(gstart))
    assert np.allclose(gstart, ostart, rtol=1e-6, atol=1e-9)
    assert np.allclose(gmom, omom, rtol=1e-6, atol=1e-9)
    # errors at the truth
    err = G.gm_param_errors(gm, db, b.truth).cpu().numpy()
    for g in range(b.n):
        re = O.param_errors(om, b.image(b.data, g), b.image(b.sigma, g), b.psf_of(g), b.truth[g])
        assert np.allclose(err[g], re, rtol=1e-4, atol=0), g
    # fits, each side from its own start
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, gstart)]
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, ostart)
    assert np.all(np.isfinite(gc)) and np.all(gs != G.ST_NONFINITE)
    npass, nboth, fails, counts = judge_batch(b, om, names, gp, gc, gs, rp, rc, rs)
    print(f"faulty pixels: parity {npass}/{nboth} {counts}; status gpu {np.bincount(gs, minlength=4).tolist()} "
          f"oracle {np.bincount(rs, minlength=4).tolist()}", flush=True)
    assert nboth >= 0.8 * b.n and npass == nboth


def test_nonfinite_start_vectors():
    b = oracle_batch("sersic64", 10, seed=62)
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    names = S.MODEL_SPECS[b.model]["names"]
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    start = ostart.copy()
    nan, inf = np.nan, np.inf
    cases = [("x0", nan), ("mag", nan), ("n", nan), ("sky", nan), ("pa", nan),
             ("mag", -inf), ("pa", -inf), ("x0", inf), ("re", inf), ("n", inf)]
    for g, (nm, v) in enumerate(cases):
        start[g, names.index(nm)] = v
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, _dev(b), start)]
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, start)
    print(f"non-finite starts: gpu status {gs.tolist()} iters {gn.tolist()}; oracle status {rs.tolist()} "
          f"iters {rn.tolist()}", flush=True)
    assert np.array_equal(gs, rs)
    assert np.all(gs[:7] == G.ST_NONFINITE) and np.all(gn[:7] == 0) and np.all(rn[:7] == 0)
    assert np.all(gs[7:] != G.ST_NONFINITE)
    # the clamped starts: equal on both sides (no trial made)
    b3 = b.subset(range(7, 10))
    gp0 = G.gm_fit_batch(gm, _dev(b3), start[7:], max_iter=0)[0].cpu().numpy()
    rp0 = O.fit_batch(om, b3.h, b3.w, b3.img_off, b3.data, b3.sigma, b3.psf_k, b3.psf_off, b3.psf, start[7:],
                      max_iter=0)[0]
    assert np.allclose(gp0, rp0, rtol=1e-12, atol=1e-12)
    assert gp0[0, names.index("x0")] == b.w[7] and abs(gp0[1, names.index("re")] - 2.0 * max(b.h[8], b.w[8])) < 1e-9
    assert abs(gp0[2, names.index("n")] - 10.0) < 1e-12
    # the fits from the clamped scale and index: parity.  The centre clamped to the
    # cutout's edge (galaxy 7) starts where the model barely overlaps the galaxy and
    # the LM path depends on rounding; its start is checked above, not its end
    b2 = b.subset(range(8, 10))
    npass, nboth, fails, counts = judge_batch(b2, om, names, gp[8:], gc[8:], gs[8:], rp[8:], rc[8:], rs[8:])
    assert nboth == 2 and npass == nboth, fails


def test_boxiness_start_outside_bounds_is_clamped():
    b = oracle_box_batch("sersic64", 6, seed=63)
    om = from_spec("sersic_box")
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic_box"])
    names = S.MODEL_SPECS["sersic_box"]["names"]
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    start = ostart.copy()
    start[:, names.index("box")] = [3.0, -2.0, 2.5, -1.5, 10.0, -0.95]
    # no trial: both sides return the clamped start and its chi^2
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, _dev(b), start, max_iter=0)]
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, start,
                                 max_iter=0)
    assert np.array_equal(gs, rs) and np.all(gn == 0) and np.all(rn == 0)
    assert np.allclose(gp, rp, rtol=1e-12, atol=1e-12)
    assert np.array_equal(gp[:, names.index("box")], [2.0, -0.9, 2.0, -0.9, 2.0, -0.9])
    assert np.allclose(gc, rc, rtol=1e-7, atol=0)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, _dev(b), start)]
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, start)
    npass, nboth, fails, counts = judge_batch(b, om, names, gp, gc, gs, rp, rc, rs)
    print(f"out-of-bounds boxiness starts: parity {npass}/{nboth} {counts}", flush=True)
    assert npass == nboth and nboth >= 3
