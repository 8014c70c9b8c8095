"""Launch schedules: every compiled plane-group variant and workgroups-per-CU
setting gives fits within the parity bar of the oracle (both from the
oracle's moment start); with one workgroup per fit the grid size does not
change a galaxy's result; the tuner picks, applies and caches a schedule."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from paper_2404_07780_amd import tune as T
from tests.gpu_helpers import judge_batch, oracle_batch
from tests.oracle_models import from_spec


def _dev(b):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf)


@pytest.mark.parametrize("cfg,n", [("sersic64", 24), ("uneven", 6), ("bulgedisk", 3)])
def test_every_schedule_matches_oracle(cfg, n):
    b = oracle_batch(cfg, n, seed=21)
    om = from_spec(b.model)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    names = S.MODEL_SPECS[b.model]["names"]
    db = _dev(b)
    ctx = G.Context()
    k = T.batch_psf_side(db)
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, ostart)
    opts = G.gm_schedule_options(gm, int(b.psf_k.max()))
    assert opts
    for ng in opts:
        res = {}
        for wpc in (0, 1):
            G.gm_set_schedule(gm, k, ng, wpc, team=1, ctx=ctx)     # one workgroup per fit
            res[wpc] = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, ostart, ctx=ctx)]
        for a, c in zip(res[0], res[1]):
            assert np.array_equal(a, c), (cfg, ng)
        gp, gc, gn, gs = res[0]
        npass, nboth, fails, counts = judge_batch(b, om, names, gp, gc, gs, rp, rc, rs)
        print(f"{cfg} plane groups {ng}: parity {npass}/{nboth} {counts} {fails}, iters {gn.mean():.2f} "
              f"(oracle {rn.mean():.2f})", flush=True)
        assert nboth >= 0.7 * b.n and npass == nboth
    ctx.close()


def test_unknown_plane_group_count_is_rejected():
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    with pytest.raises(G.GmError) as e:
        G.gm_set_schedule(gm, 15, 7, 0, ctx=G.Context())
    assert e.value.code == G.GM_EUNSUPPORTED


def test_tuner_applies_and_caches(tmp_path):
    b = oracle_batch("sersic64", 64, seed=22)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    db = _dev(b)
    ctx = G.Context()
    path = str(tmp_path / "tune.json")
    r1 = T.apply(gm, db, cache_path=path, sample=64, ctx=ctx)
    # plane groups x residency, then workgroups per fit (one each: the 64-galaxy sample forms teams by default)
    assert not r1["cached"] and len(r1["trials"]) == 2 * len(G.gm_schedule_options(gm, 15)) + 1
    assert {t["team"] for t in r1["trials"]} == {0, 1}
    cache = json.load(open(path))
    assert r1["key"] in cache and cache[r1["key"]]["plane_groups"] == r1["plane_groups"]
    assert cache[r1["key"]]["team"] == r1["team"]
    r2 = T.apply(gm, db, cache_path=path, ctx=ctx)
    assert r2["cached"] and r2["plane_groups"] == r1["plane_groups"]
    print(f"tuned {r1['key']}: {r1['trials']}", flush=True)
    ctx.close()
