"""Pins of the fit-parity judge (tests/gpu_helpers.judge_fit) on the oracle
alone: two oracle fits of the same data from different starts.

- A nearly round galaxy: its position angle is not determined by the data
  (covariance error of hundreds of degrees), and two fits that both pass the
  stop test differ in PA by far more than 1e-4 of its value while every
  parameter stays within 2 step_tol sigma of the other fit.  The judge takes
  such a pair as one result ("sigma"); a planted offset of a few step_tol
  sigma, or a centre moved by a small fraction of its error, fails.
- A centre next to an integer row boundary: the oversampled central window
  sits at row floor(H - y0), so chi^2 has a step where that floor changes,
  and the oracle itself converges to one minimum on each side, depending on
  the start.  The judge takes the pair as two results of the method ("hop");
  a point moved across the boundary without being a minimum there fails the
  oracle's stop test and is rejected.
"""
import numpy as np
import pytest

import oracle as O
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import judge_fit, oracle_batch, param_parity
from tests.oracle_models import from_spec

NAMES = S.MODEL_SPECS["sersic"]["names"]
IPA, IY0 = NAMES.index("pa"), NAMES.index("y0")


def _galaxy(index):
    """Galaxy `index` of the held-out single-Sersic 64 x 64 draw (seed 2),
    rendered by the oracle and noised on the host, and the oracle's fit from
    its moment start."""
    b = oracle_batch("sersic64", 1, seed=2, start=index)
    om = from_spec(b.model)
    d, s, psf = b.image(b.data, 0), b.image(b.sigma, 0), b.psf_of(0)
    start, _ = O.default_guess(om, d, s)
    rp, rc, rn, rs = O.fit(om, d, s, psf, start)
    assert rs == 0
    return om, d, s, psf, start, rp, rc


@pytest.fixture(scope="module")
def round_galaxy():
    om, d, s, psf, start, rp, rc = _galaxy(1596)
    assert rp[NAMES.index("q")] > 0.999
    return om, d, s, psf, start, rp, rc


def test_round_galaxy_position_angle_in_sigma_units(round_galaxy):
    om, d, s, psf, start, rp, rc = round_galaxy
    err = O.param_errors(om, d, s, psf, rp)
    assert err[IPA] > 1000.0                     # PA undetermined
    verdicts = []
    for dpa in (30.0, 90.0):
        st = start.copy()
        st[IPA] += dpa
        p2, c2, n2, s2 = O.fit(om, d, s, psf, st)
        assert s2 == 0
        ok_rel, worst = param_parity(NAMES, p2, rp, sky_sigma=float(np.median(s)))
        assert not ok_rel.all() and worst[IPA] > 10.0    # the relative bar cannot hold for PA
        ok, how, _ = judge_fit(om, NAMES, d, s, psf, p2, rp, c2, rc)
        verdicts.append(how)
        assert ok and how == "sigma"
    print(f"round galaxy verdicts {verdicts}")


def test_sigma_rule_rejects_planted_offsets(round_galaxy):
    om, d, s, psf, start, rp, rc = round_galaxy
    err = O.param_errors(om, d, s, psf, rp)
    # PA moved by 5 step_tol sigma: beyond the 2 step_tol sigma reach of the stop test
    bad = rp.copy()
    bad[IPA] += 5e-4 * err[IPA]
    assert judge_fit(om, NAMES, d, s, psf, bad, rp)[0] is False
    # PA moved by 1 step_tol sigma: inside it
    near = rp.copy()
    near[IPA] += 1e-4 * err[IPA]
    assert judge_fit(om, NAMES, d, s, psf, near, rp)[1] == "sigma"
    # a well-determined parameter moved by 1e-2 of its error (beyond both bars)
    for k in (NAMES.index("x0"), NAMES.index("re"), NAMES.index("sky")):
        bad = rp.copy()
        bad[k] += 1e-2 * err[k] + 2e-4 * max(abs(rp[k]), 1.0)
        assert judge_fit(om, NAMES, d, s, psf, bad, rp)[0] is False, NAMES[k]


@pytest.fixture(scope="module")
def boundary_galaxy():
    om, d, s, psf, start, rp, rc = _galaxy(1202)
    assert abs(rp[IY0] - 31.0) < 2e-3
    return om, d, s, psf, start, rp, rc


def test_window_step_pair_is_two_results(boundary_galaxy):
    om, d, s, psf, start, rp, rc = boundary_galaxy
    h = d.shape[0]
    st = rp.copy()
    st[IY0] = 2.0 * np.round(rp[IY0]) - rp[IY0]        # mirror the centre across the boundary
    p2, c2, n2, s2 = O.fit(om, d, s, psf, st)
    assert s2 == 0
    assert np.floor(h - p2[IY0]) != np.floor(h - rp[IY0])      # the two ends straddle the boundary
    assert abs(c2 - rc) < 1.0 and abs(c2 - rc) > 1e-6            # two distinct minima
    assert not param_parity(NAMES, p2, rp, sky_sigma=float(np.median(s)))[0].all()
    ok, how, _ = judge_fit(om, NAMES, d, s, psf, p2, rp, c2, rc)
    assert ok and how == "hop"


def test_window_step_needs_a_minimum(boundary_galaxy):
    om, d, s, psf, start, rp, rc = boundary_galaxy
    for dy in (1e-2, 5e-3):            # beyond the 1e-4 relative bar of y0 (3.1e-3 px)
        moved = rp.copy()
        moved[IY0] = np.round(rp[IY0]) - dy            # across the boundary, not refitted
        ok, how, _ = judge_fit(om, NAMES, d, s, psf, moved, rp, rc, rc)
        assert not ok and how == "fail", dy
