"""Captured plans (gm_plan_fit, gm_plan_fit_learned): every graph replay gives
the eager calls' results (fit with its covariance errors) bit for bit -- the same kernels run on the same
inputs -- including replays separated by other eager work on the parent
context (which grows and overwrites its own workspace) and by changes of the
plan's inputs.  The eager calls themselves are held to the oracle by the
parity tests."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import mlp as M
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import learned as Lrn
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import oracle_batch


def _dev(b):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf, omega=b.omega)


def _np(*ts):
    return [t.cpu().numpy() for t in ts]


def _same(a, b):
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


def _other_eager_work(ctx):
    """A bigger fit on the parent context between replays, plus torch work."""
    b = oracle_batch("uneven", 6, seed=31)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    db = _dev(b)
    start, _ = G.gm_default_guess(gm, db, ctx=ctx)
    G.gm_fit_batch(gm, db, start, ctx=ctx, max_iter=5)
    x = torch.randn(1 << 20, device="cuda")
    (x * 2.0).sum().item()
    torch.cuda.synchronize()


@pytest.mark.parametrize("cfg,n,with_start", [("sersic64", 40, False), ("sersic64", 40, True),
                                              ("uneven", 10, False), ("bulgedisk", 6, True)])
def test_plan_fit_replays_equal_eager(cfg, n, with_start):
    print(f"plan fit {cfg} n={n} start={'given' if with_start else 'moments'}", flush=True)
    b = oracle_batch(cfg, n, seed=21)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    ctx = G.Context()
    db = _dev(b)
    guess, _ = G.gm_default_guess(gm, db, ctx=ctx)
    start = guess.clone() if with_start else None
    if with_start:
        start[:, 0] += 0.3          # a start that is not the moment guess
    plan = G.gm_plan_fit(gm, db, start=start, errors=True, ctx=ctx)

    def eager():
        p0 = start.clone() if with_start else G.gm_default_guess(gm, db, ctx=ctx)[0]
        err = torch.empty(b.n, gm.p, dtype=torch.float64, device="cuda")
        p, c, it, st = G.gm_fit_batch(gm, db, p0, ctx=ctx, err_out=err)
        return _np(p, c, it, st, err)

    ref = eager()
    for rep in range(3):
        plan.launch()
        torch.cuda.synchronize()
        got = _np(plan.params, plan.chi2, plan.niter, plan.status, plan.err)
        assert _same(got, ref), (cfg, rep)
        _other_eager_work(ctx)
    if with_start:
        # the plan reads the caller's start buffer in place: new contents are
        # used by the next launch
        start[:, 1] -= 0.2
        ref2 = eager()
        plan.launch()
        torch.cuda.synchronize()
        assert _same(_np(plan.params, plan.chi2, plan.niter, plan.status, plan.err), ref2)
    plan.close()
    ctx.close()


def test_plan_fit_learned_replays_equal_eager():
    b = oracle_batch("sersic64", 48, seed=22)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    db = _dev(b)
    ctx = G.Context()
    # a network that proposes the moments (n = e^0.6): some proposals converge,
    # the budget of 10 trials sends the rest to the fallback
    mlp = G.MLP(np.zeros(M.param_count(), np.float32), train=False)
    plan = G.gm_plan_fit_learned(gm, db, mlp, proposal_max_iter=10, errors=True, ctx=ctx)
    err = torch.empty(b.n, gm.p, dtype=torch.float64, device="cuda")
    p, c, it, st, fb = G.gm_fit_learned(gm, db, mlp, proposal_max_iter=10, ctx=ctx, err_out=err)
    ref = _np(p, c, it, st, fb, err)
    print(f"learned plan: fallback codes {np.bincount(ref[4], minlength=3).tolist()}", flush=True)
    assert (ref[4] == 0).any() and (ref[4] == 2).any()
    for rep in range(3):
        plan.launch()
        torch.cuda.synchronize()
        got = _np(plan.params, plan.chi2, plan.niter, plan.status, plan.fallback, plan.err)
        assert _same(got, ref), rep
        _other_eager_work(ctx)
    # new weights in the same buffers are used by the next launch
    flat = Lrn.init_params(3)
    mlp.params.copy_(torch.from_numpy(flat).to(mlp.params.device))
    G.gm_mlp_sync(mlp, ctx=ctx)
    p, c, it, st, fb = G.gm_fit_learned(gm, db, mlp, proposal_max_iter=10, ctx=ctx)
    ref2 = _np(p, c, it, st, fb)
    plan.launch()
    torch.cuda.synchronize()
    assert _same(_np(plan.params, plan.chi2, plan.niter, plan.status, plan.fallback), ref2)
    plan.close()
    ctx.close()


def test_plan_events_time_the_lm_launch():
    b = oracle_batch("sersic64", 64, seed=23)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    db = _dev(b)
    plan = G.gm_plan_fit(gm, db, errors=True, timing=True)
    with pytest.raises(G.GmError):
        plan.elapsed()                 # not launched yet
    for _ in range(2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.launch()
        e1.record()
        ms = plan.elapsed()
        torch.cuda.synchronize()
        total = e0.elapsed_time(e1)
        print(f"plan events: guess {ms[0]:.3f} LM {ms[1]:.3f} errors {ms[2]:.3f} ms of {total:.3f} ms", flush=True)
        assert all(v > 0.0 for v in ms) and sum(ms) <= total * 1.001 + 0.01
    untimed = G.gm_plan_fit(gm, db, errors=False)
    untimed.launch()
    with pytest.raises(G.GmError):
        untimed.elapsed()


def test_plan_rejects_bad_arguments():
    b = oracle_batch("sersic64", 2, seed=24)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    db = _dev(b)
    with pytest.raises(G.GmError):
        G.gm_plan_fit(gm, db, max_iter=-1)
    empty = G.Batch(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), np.zeros(0, np.int32),
                    np.zeros(0, np.int64), np.zeros(1, np.float32), np.ones(1, np.float32), np.ones(1, np.float32))
    with pytest.raises(G.GmError):
        G.gm_plan_fit(gm, empty)
