"""gm_fit_batch_noalloc, the fit entry point for callers that cannot
allocate, through the C ABI: its results equal gm_fit_batch's bit for bit
when that runs one workgroup per fit too (same kernels, per-galaxy results
independent of the fit order) on two calls in a row, the second with a
smaller batch (the library's fixed device array keeps the first call's
contents, which must not leak into the second); and a batch above the
array's limit is rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import oracle_batch


def _dev(b):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf, omega=b.omega)


def _both(b, gm, ctx, err=False):
    db = _dev(b)
    start, _ = G.gm_default_guess(gm, db, ctx=ctx)
    e1 = torch.empty(b.n, gm.p, dtype=torch.float64, device="cuda") if err else None
    ref = G.gm_fit_batch(gm, db, start, err_out=e1, ctx=ctx)
    params = start.clone()
    chi2 = torch.full((b.n,), -1.0, dtype=torch.float64, device="cuda")
    niter = torch.full((b.n,), -1, dtype=torch.int32, device="cuda")
    status = torch.full((b.n,), -1, dtype=torch.int32, device="cuda")
    e2 = torch.empty(b.n, gm.p, dtype=torch.float64, device="cuda") if err else None
    G.gm_fit_batch_noalloc(gm, db, params, chi2, niter, status, err_out=e2, ctx=ctx)
    for a, c in zip(ref, (params, chi2, niter, status)):
        assert torch.equal(a, c)
    if err:
        assert torch.equal(e1, e2)
    return status.cpu().numpy()


def test_noalloc_equals_fit_batch_on_two_calls():
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    ctx = G.Context()
    for k in (15, 25):
        G.gm_set_schedule(gm, k, team=1, ctx=ctx)     # one workgroup per fit, as the no-alloc variant runs
    print("no-alloc fit: uneven sizes, 40 galaxies, then sersic64, 12 galaxies", flush=True)
    st1 = _both(oracle_batch("uneven", 40, seed=91), gm, ctx, err=True)
    st2 = _both(oracle_batch("sersic64", 12, seed=92), gm, ctx)
    ctx.close()
    print(f"statuses {np.bincount(st1, minlength=4).tolist()} then {np.bincount(st2, minlength=4).tolist()}",
          flush=True)


def test_noalloc_rejects_batches_above_its_limit():
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    n = G.NOALLOC_MAX_GAL + 1
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    psf = torch.ones(1, dtype=torch.float32, device="cuda")
    db = G.Batch(np.ones(n), np.ones(n), np.arange(n), np.ones(n), np.zeros(n), ones, ones, psf)
    params = torch.zeros(n, gm.p, dtype=torch.float64, device="cuda")
    chi2 = torch.empty(n, dtype=torch.float64, device="cuda")
    niter = torch.empty(n, dtype=torch.int32, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(G.GmError) as e:
        G.gm_fit_batch_noalloc(gm, db, params, chi2, niter, status)
    assert e.value.code == G.GM_EINVAL
