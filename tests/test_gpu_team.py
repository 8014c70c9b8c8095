"""Fits shared by teams of workgroups (gm_schedule.team) against the FP64
oracle.

A launch with fewer fits than resident workgroups gives each fit several
workgroups by default (the paper's Sec. 7: small batches leave the GPU idle);
each shares the model evaluations tile by tile and the leader adds their FP64
partial sums in a fixed order.  The fits are the same method, so they are
judged against the oracle with the parity bar of the other fit tests
(tests/gpu_helpers.judge_fit), and against one-workgroup fits at that bar
(only the last bits of the sums differ).  Cases: the 64-galaxy 64 x 64
workload (teams of 4), 8 galaxies of 1024 x 1024 (teams of up to 32), teams
only for the largest cutouts of an uneven batch, reproducibility, and waits
forced past a tiny limit from the host (every fit then ends, with
GM_ST_TEAM_TIMEOUT or normally)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import judge_batch, oracle_batch
from tests.oracle_models import from_spec


def _dev(b):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf, omega=b.omega)


def _timed_fit(gm, db, start, ctx, reps=3):
    out = G.gm_fit_batch(gm, db, start, ctx=ctx)        # warm-up (and the result)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        G.gm_fit_batch(gm, db, start, ctx=ctx)
    ev[1].record()
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out], ev[0].elapsed_time(ev[1]) / reps


def _team_vs_single(b, ctx_team, ctx_one):
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    names = S.MODEL_SPECS[b.model]["names"]
    db = _dev(b)
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    (tp, tc, tn, ts), ms_team = _timed_fit(gm, db, ostart, ctx_team)
    (sp, sc, sn, ss), ms_one = _timed_fit(gm, db, ostart, ctx_one)
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, ostart)
    npass, nboth, fails, counts = judge_batch(b, om, names, tp, tc, ts, rp, rc, rs)
    # team against one workgroup: the same method, sums differing in their last bits
    npass1, nboth1, fails1, _ = judge_batch(b, om, names, tp, tc, ts, sp, sc, ss)
    print(f"  teams {ms_team:.2f} ms vs one workgroup per fit {ms_one:.2f} ms ({ms_one / ms_team:.2f}x; "
          f"{b.n / ms_team * 1e3:.0f} vs {b.n / ms_one * 1e3:.0f} galaxies/s); oracle parity {npass}/{nboth} "
          f"{counts} {fails}; team vs one {npass1}/{nboth1} {fails1}; status {np.bincount(ts, minlength=5).tolist()}",
          flush=True)
    assert nboth >= 0.6 * b.n and npass == nboth
    assert npass1 == nboth1 and nboth1 >= 0.6 * b.n
    return ms_team, ms_one


@pytest.fixture()
def ctxs():
    ctx_team, ctx_one = G.Context(), G.Context()
    yield ctx_team, ctx_one
    ctx_team.close()
    ctx_one.close()


def _one_per_fit(gm, ctx):
    for k in (0, 15, 25):
        G.gm_set_schedule(gm, k, team=1, ctx=ctx)


def test_small_batch_teams(ctxs):
    """64 galaxies of 64 x 64 (4 tiles): teams of 4 by default."""
    print("teams: sersic64, 64 galaxies", flush=True)
    b = oracle_batch("sersic64", 64, seed=0)
    _one_per_fit(G.Model.from_spec(S.MODEL_SPECS[b.model]), ctxs[1])
    ms_team, ms_one = _team_vs_single(b, *ctxs)
    assert ms_team < ms_one


def test_large_cutout_teams(ctxs):
    """8 galaxies of 1024 x 1024 (1024 tiles each): teams of up to 32."""
    print("teams: 8 galaxies of 1024 x 1024", flush=True)
    rng = np.random.default_rng(95)
    n, H = 8, 1024
    psf = S.gaussian_psf(1.5, 15)
    truth = np.column_stack([512 + rng.uniform(-2, 2, n), 512 + rng.uniform(-2, 2, n), rng.uniform(11, 13, n),
                             rng.uniform(20, 60, n), rng.uniform(0.8, 3.0, n), rng.uniform(0.4, 0.9, n),
                             rng.uniform(0, 180, n), rng.uniform(50, 100, n)])
    om = from_spec("sersic")
    data = np.concatenate([(O.model_image(om, H, H, psf, truth[g]) + rng.normal(size=(H, H))).ravel()
                           for g in range(n)]).astype(np.float32)
    hs = np.full(n, H, np.int32)
    b = S.Batch("sersic64", "sersic", hs, hs.copy(), np.arange(n, dtype=np.int64) * H * H, np.full(n, 15, np.int32),
                np.arange(n, dtype=np.int64) * psf.size, np.tile(psf.ravel(), n).astype(np.float32), truth,
                np.ones(n), np.ones(n), np.arange(n))
    b.data = data
    b.sigma = np.ones(b.npix, np.float32)
    _one_per_fit(G.Model.from_spec(S.MODEL_SPECS["sersic"]), ctxs[1])
    ms_team, ms_one = _team_vs_single(b, *ctxs)
    assert ms_team < ms_one


def test_teams_for_the_largest_cutouts_only():
    """An uneven batch with teams of up to 4 for fits of at least 16 tiles."""
    print("teams: uneven sizes, teams of 4 for cutouts of >= 16 tiles", flush=True)
    b = oracle_batch("uneven", 16, seed=96)
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    names = S.MODEL_SPECS[b.model]["names"]
    ctx = G.Context()
    G.gm_set_schedule(gm, 25, team=4, team_min_tiles=16, ctx=ctx)
    db = _dev(b)
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, ostart, ctx=ctx)]
    again = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, ostart, ctx=ctx)]
    for a, c in zip((gp, gc, gn, gs), again):
        assert np.array_equal(a, c)                    # fixed-order sums: reproducible
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, ostart)
    npass, nboth, fails, counts = judge_batch(b, om, names, gp, gc, gs, rp, rc, rs)
    tiles = ((b.h + 31) // 32) * ((b.w + 31) // 32)
    print(f"  {int((tiles >= 16).sum())} of {b.n} fits in teams; parity {npass}/{nboth} {counts} {fails}", flush=True)
    assert (tiles >= 16).any() and (tiles < 16).any()
    assert nboth >= 0.8 * b.n and npass == nboth
    ctx.close()


def test_team_waits_past_their_limit_end_the_fit():
    """Waits bounded at 1 us (forced from the host): every fit of the launch
    ends, the ones whose team missed the bound with GM_ST_TEAM_TIMEOUT; the
    same context then fits normally with the default bound."""
    print("teams: waits bounded at 1 us", flush=True)
    b = oracle_batch("sersic64", 16, seed=97)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    db = _dev(b)
    ctx = G.Context()
    G.gm_set_schedule(gm, 15, team=4, team_wait_us=1, ctx=ctx)
    start, _ = G.gm_default_guess(gm, db, ctx=ctx)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start, ctx=ctx)]
    print(f"  statuses with a 1 us bound: {np.bincount(gs, minlength=5).tolist()}", flush=True)
    assert set(np.unique(gs)) <= {G.ST_CONVERGED, G.ST_MAXITER, G.ST_STALLED, G.ST_TEAM_TIMEOUT}
    assert (gs == G.ST_TEAM_TIMEOUT).any()
    G.gm_set_schedule(gm, 15, team=4, ctx=ctx)
    gp2, gc2, gn2, gs2 = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start, ctx=ctx)]
    assert not (gs2 == G.ST_TEAM_TIMEOUT).any() and (gs2 == G.ST_CONVERGED).mean() >= 0.8
    ctx.close()
