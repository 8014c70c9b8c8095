"""Autotuner of the fitting kernels' launch schedule.

For a model and a batch, every plane-group count compiled for the model's
family (gm_schedule_options) is tried with the persistent grid at full
residency and at one workgroup per CU: the LM fit from the moment start runs
on a sample of the batch under each schedule (gm_set_schedule) and the
fastest is kept.  By default each galaxy of a sample gets a fixed number of
trials, so that every schedule does the same work and the time measures the
throughput per evaluation rather than the few slowest fits of the sample;
with trials=0 the fits run to completion, which also measures how a schedule
copes with the slowest fits (it matters for batches of very uneven cutouts,
where the largest fits that need the most trials finish last and run at half
speed when two workgroups share a CU).  Results are cached in a JSON file keyed by
(device architecture, family, PSF side, parameter count, cutout-size bucket),
so later runs apply a known schedule without timing.

A second stage then tries workgroups per fit (gm_schedule.team) on top of the
best plane-group count and residency: one workgroup per fit when the sample
is small enough for the automatic teams to form, and teams of 2 or 4 for the
fits of at least 16 tiles (128 x 128 px) when the batch has such cutouts, so
that the largest fits of an uneven batch end sooner.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional

import numpy as np
import torch

from . import gmfit as G


def family_key(model: G.Model) -> str:
    parts = []
    for c in model.comps:
        parts.append(f"{c.type}{'c' if c.convolve else 'u'}")
    return "+".join(parts)


def size_bucket(batch: G.Batch) -> int:
    """log2 of the mean cutout area, rounded."""
    return int(round(math.log2(max(float(np.mean(batch.h.astype(np.float64) * batch.w)), 1.0))))


def batch_psf_side(batch: G.Batch) -> int:
    ks = np.unique(batch.psf_k)
    return int(ks[0]) if len(ks) == 1 else 0


def cache_key(model: G.Model, batch: G.Batch) -> str:
    arch = torch.cuda.get_device_properties(batch.device).gcnArchName.split(":")[0]
    return f"{arch}|{family_key(model)}|K{batch_psf_side(batch)}|p{model.p}|a{size_bucket(batch)}"


def subset(batch: G.Batch, n: int) -> G.Batch:
    """The first n galaxies, sharing the device pixels (offsets unchanged)."""
    n = min(n, batch.n)
    return G.Batch(batch.h[:n], batch.w[:n], batch.img_off[:n], batch.psf_k[:n], batch.psf_off[:n], batch.data,
                   batch.sigma, batch.psf, omega=batch.omega, device=batch.device)


def _time_fit(model, sb, start, ctx, reps: int, trials: int) -> float:
    mi = trials if trials > 0 else 100
    G.gm_fit_batch(model, sb, start, ctx=ctx, max_iter=mi)      # warm-up (kernel load, workspace growth)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        G.gm_fit_batch(model, sb, start, ctx=ctx, max_iter=mi)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(model: G.Model, batch: G.Batch, sample: int = 4096, reps: int = 3, trials: int = 4,
         ctx: Optional[G.Context] = None) -> Dict:
    """Time every schedule on the first `sample` galaxies with `trials` LM trials
    each (0: complete fits), apply the fastest and return {"plane_groups",
    "wg_per_cu", "ms", "trials" (every schedule's time)}."""
    ctx = ctx or G.context(batch.device.index)
    k = batch_psf_side(batch)
    sb = subset(batch, sample)
    start, _ = G.gm_default_guess(model, sb, ctx=ctx)
    results = []
    for ng in G.gm_schedule_options(model, k if k else int(batch.psf_k.max())):
        for wpc in (0, 1):
            G.gm_set_schedule(model, k, ng, wpc, ctx=ctx)
            results.append(dict(plane_groups=ng, wg_per_cu=wpc, team=0, team_min_tiles=0,
                                ms=_time_fit(model, sb, start, ctx, reps, trials)))
    best = min(results, key=lambda t: t["ms"])
    tiles = ((sb.h.astype(np.int64) + 31) // 32) * ((sb.w.astype(np.int64) + 31) // 32)
    teams = []
    if sb.n <= 2048:
        teams.append((1, 0))
    if (tiles >= 16).any():
        teams += [(2, 16), (4, 16)]
    for team, tmin in teams:
        G.gm_set_schedule(model, k, best["plane_groups"], best["wg_per_cu"], team=team, team_min_tiles=tmin, ctx=ctx)
        results.append(dict(plane_groups=best["plane_groups"], wg_per_cu=best["wg_per_cu"], team=team,
                            team_min_tiles=tmin, ms=_time_fit(model, sb, start, ctx, reps, trials)))
    best = min(results, key=lambda t: t["ms"])
    G.gm_set_schedule(model, k, best["plane_groups"], best["wg_per_cu"], team=best["team"],
                      team_min_tiles=best["team_min_tiles"], ctx=ctx)
    return dict(best, trials=results, sample=sb.n, trials_per_galaxy=trials)


def load(path: str) -> Dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(path: str, cache: Dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(model: G.Model, batch: G.Batch, cache_path: Optional[str] = None, sample: int = 4096, trials: int = 4,
          ctx: Optional[G.Context] = None) -> Dict:
    """Apply the cached schedule for this model and batch, tuning (and caching,
    when a path is given) if there is none."""
    ctx = ctx or G.context(batch.device.index)
    key = cache_key(model, batch)
    cache = load(cache_path) if cache_path else {}
    if key in cache:
        e = cache[key]
        G.gm_set_schedule(model, batch_psf_side(batch), e["plane_groups"], e["wg_per_cu"], team=e.get("team", 0),
                          team_min_tiles=e.get("team_min_tiles", 0), ctx=ctx)
        return dict(e, key=key, cached=True)
    res = tune(model, batch, sample=sample, trials=trials, ctx=ctx)
    if cache_path:
        cache[key] = {k: res[k] for k in ("plane_groups", "wg_per_cu", "team", "team_min_tiles", "ms")}
        save(cache_path, cache)
    return dict(res, key=key, cached=False)
