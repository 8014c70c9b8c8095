"""Parity at full size, in the launch configuration the benchmark times: the
whole batch of a workload is fitted in one persistent launch, and sampled
galaxies spread over the batch are checked against the FP64 oracle.  The
sampled galaxies' images are rendered by the oracle and noised on the host;
the rest of the batch (rendered by the HIP forward model) only fills the
launch and is not judged, so no oracle input comes from the GPU."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import learned as Lrn
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import judge_fit
from tests.oracle_models import from_spec


def _full_batch(cfg, n, seed, sample):
    """Draw n galaxies; units from the HIP model except the sampled ones,
    rendered by the oracle; host noise for all."""
    b = S.draw(cfg, n, seed=seed)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    om = from_spec(b.model)
    ut = S.unit_truth(b)
    zeros = torch.zeros(b.npix, dtype=torch.float32, device="cuda")
    db = G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, zeros, zeros, b.psf)
    units = G.gm_model_image(gm, db, ut).cpu().numpy().astype(np.float64)
    for g in sample:
        h, w, o = int(b.h[g]), int(b.w[g]), int(b.img_off[g])
        units[o:o + h * w] = O.model_image(om, h, w, b.psf_of(g), ut[g]).ravel()
    S.finish(b, units)
    return b, gm, om, G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf)


def _judge(b, om, names, sample, gp, gc, gs):
    """judge_fit of the sampled galaxies that both sides converge, the oracle
    fitting each from its own moment start."""
    npass = nboth = 0
    fails, counts = [], {}
    for g in sample:
        data, sigma = b.image(b.data, g), b.image(b.sigma, g)
        start, _ = O.default_guess(om, data, sigma)
        rp, rc, rn, rs = O.fit(om, data, sigma, b.psf_of(g), start)
        if rs != 0 or gs[g] != 0:
            continue
        nboth += 1
        ok, how, worst = judge_fit(om, names, data, sigma, b.psf_of(g), gp[g], rp, gc[g], rc)
        counts[how] = counts.get(how, 0) + 1
        if ok:
            npass += 1
        else:
            fails.append((int(g), round(worst, 2)))
    print(f"  verdicts {counts}", flush=True)
    return npass, nboth, fails


def test_uneven_8192_one_launch():
    n = 8192
    sample = np.linspace(0, n - 1, 24).astype(int)
    print(f"uneven: {n} galaxies, sampled {sample.tolist()}", flush=True)
    b, gm, om, db = _full_batch("uneven", n, 0, sample)
    start, _ = G.gm_default_guess(gm, db)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start)]
    npass, nboth, fails = _judge(b, om, S.MODEL_SPECS[b.model]["names"], sample, gp, gc, gs)
    print(f"uneven full launch: converged {np.mean(gs == 0):.4f}; sampled parity {npass}/{nboth} {fails}", flush=True)
    assert nboth >= 0.8 * len(sample) and npass == nboth


def test_learned_65536_one_launch():
    n = 65536
    sample = np.linspace(0, n - 1, 32).astype(int)
    print("training a proposal network on 65536 forward-model galaxies (4 epochs)", flush=True)
    ds = Lrn.make_training_set(65536, seed=1)
    mlp = Lrn.new_mlp(0)
    Lrn.train(mlp, ds, epochs=4, batch=4096)
    del ds
    print(f"learned: {n} galaxies, sampled {sample.tolist()}", flush=True)
    b, gm, om, db = _full_batch("sersic64", n, 2, sample)
    lp, lc, ln, ls, fb = [t.cpu().numpy() for t in G.gm_fit_learned(gm, db, mlp)]
    npass, nboth, fails = _judge(b, om, S.MODEL_SPECS[b.model]["names"], sample, lp, lc, ls)
    print(f"learned full launch: converged {np.mean(ls == 0):.4f}, refitted {int((fb != 0).sum())}; "
          f"sampled parity {npass}/{nboth} {fails}", flush=True)
    assert nboth >= 0.8 * len(sample) and npass == nboth
