"""Learned proposal on the GPU against the oracle (oracle/mlp.py, orc_moments,
the LM oracle) and the test-side Philox reference.

Tolerances.  GEMMs accumulate in FP32 on the device and exactly in the oracle,
which otherwise rounds to BF16 at the same points; a rounding that lands on
the other side of a BF16 tie moves one value by one BF16 step (2^-8
relative), so network outputs are compared to 4e-3 of their scale (median 1e-5), gradients
per layer to 2e-3 in relative Frobenius norm, and features allow one BF16
step on at most 1% of the values.  Fitted parameters: 1e-4 relative (floors
in tests/gpu_helpers.py) against the oracle's LM from its own moment guess,
which judges the learned start.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O
from oracle import mlp as M
from paper_2404_07780_amd import gmfit as G
from paper_2404_07780_amd import learned as Lrn
from paper_2404_07780_amd import synth as S
from tests.gpu_helpers import judge_batch, oracle_batch, oracle_mixed, param_parity
from tests.oracle_models import from_spec
from tests.philox_ref import galaxy_normals

FULL = (1056, 512, 3, 16)


def _dev(b, omega=None):
    return G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf, omega=omega)


def _bf16_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda().to(torch.bfloat16)


def _random_params(seed, dims=FULL, n_out=7):
    flat = M.init_params(seed, *dims, n_out=n_out)
    rng = np.random.default_rng(seed + 100)
    for l, (W, b) in enumerate(M.unpack(flat, *dims)):
        b[...] = rng.normal(scale=0.05, size=b.shape).astype(np.float32)
        if l == len(M.layer_dims(*dims)) - 1:
            b[n_out:] = 0.0
    return flat


def _usable(data, sigma, omega):
    ok = np.isfinite(data) & np.isfinite(sigma) & (sigma > 0)
    return ok if omega is None else ok & (omega != 0)


@pytest.mark.parametrize("dims,n_out,n", [(FULL, 7, 200), ((64, 64, 2, 16), 3, 70), ((1056, 512, 3, 16), 7, 1)])
def test_forward_matches_oracle(dims, n_out, n):
    print(f"forward dims {dims} n {n}", flush=True)
    flat = _random_params(1, dims, n_out)
    rng = np.random.default_rng(2)
    x = M.bf16(rng.normal(size=(n, dims[0])))
    mlp = G.MLP(flat, *dims, n_out=n_out, train=False)
    assert torch.equal(mlp.params_bf16.float().cpu(), torch.from_numpy(M.bf16(flat).astype(np.float32)))
    got = G.gm_mlp_forward(mlp, _bf16_dev(x)).cpu().numpy()
    ref, _ = M.forward(flat.astype(np.float64), x, emulate_bf16=True, dims=dims)
    scale = np.abs(ref[:, :n_out]).max()
    errs = np.abs(got - ref)
    err = errs.max()
    print(f"forward max err {err:.3e}, median {np.median(errs):.3e}, of scale {scale:.3e}", flush=True)
    # one hidden activation a step of 2^-8 away moves an output by ~|w| |a| 2^-8 ~ 1e-3 of the
    # scale; FP32 accumulation alone stays near 1e-6
    assert err <= 4e-3 * scale
    assert np.median(errs) <= 1e-5 * scale
    assert np.all(got[:, n_out:] == 0.0)


def test_backward_matches_oracle():
    flat = _random_params(3)
    rng = np.random.default_rng(4)
    n = 160
    x = M.bf16(rng.normal(size=(n, 1056)))
    t = np.zeros((n, 16), np.float32)
    t[:, :7] = rng.normal(size=(n, 7))
    mlp = G.MLP(flat)
    xd = _bf16_dev(x)
    td = torch.from_numpy(t).cuda()
    loss = G.gm_mlp_backward(mlp, xd, td).item()
    grad = mlp.grad.cpu().numpy().astype(np.float64)
    rl, rg, _ = M.loss_and_grad(flat.astype(np.float64), x, t.astype(np.float64))
    assert abs(loss - rl) <= 1e-5 * rl, (loss, rl)
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(M.unpack(grad), M.unpack(rg))):
        for name, a, b in (("W", gW, rW), ("b", gb, rb)):
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
            print(f"layer {l} {name}: rel err {rel:.2e}", flush=True)
            assert rel <= 2e-3, (l, name, rel)
    # element by element: dW_l[o][i] = sum_m dZ_l[m][o] X_l[m][i] within 2^-7 of
    # sum_m |dZ_l[m][o]| |X_l[m][i]| (a BF16 rounding of one dZ or X value landing on
    # the other side of a tie moves the sum by 2^-8 of one term); an operand read
    # from a wrong row, column or tile edge moves it by a large part of that sum
    _, (acts, zs) = M.forward(flat.astype(np.float64), x, emulate_bf16=True)
    layers = M.unpack(flat.astype(np.float64))
    out, _ = M.forward(flat.astype(np.float64), x, emulate_bf16=True)
    dz = np.zeros_like(out)
    dz[:, :7] = 2.0 * (out[:, :7] - t[:, :7]) / (n * 7)
    dz = M.bf16(dz)
    for l in range(len(layers) - 1, -1, -1):
        gW, gb = M.unpack(grad)[l]
        bound = 2.0 ** -7 * (np.abs(dz).T @ np.abs(acts[l])) + 1e-30
        ratio = np.abs(gW - M.unpack(rg)[l][0]) / bound
        print(f"layer {l} W element-wise: worst {ratio.max():.3f} of the bar", flush=True)
        assert np.all(ratio <= 1.0), (l, np.unravel_index(np.argmax(ratio), ratio.shape))
        if l > 0:
            dz = M.bf16(M.bf16(dz @ M.bf16(layers[l][0])) * M.gelu_grad(zs[l - 1]))
    gW, gb = M.unpack(grad)[-1]
    assert np.all(gW[7:] == 0) and np.all(gb[7:] == 0)
    # a row gather gives exactly the gradient of the gathered rows
    rows = rng.permutation(n)[:96].astype(np.int32)
    G.gm_mlp_backward(mlp, xd, td, rows=torch.from_numpy(rows).cuda())
    g1 = mlp.grad.clone()
    G.gm_mlp_backward(mlp, _bf16_dev(x[rows]), torch.from_numpy(t[rows]).cuda())
    assert torch.equal(g1, mlp.grad)


def test_adamw_matches_oracle():
    dims = (64, 64, 1, 16)
    flat = _random_params(5, dims)
    mlp = G.MLP(flat, *dims)
    rng = np.random.default_rng(6)
    p = flat.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step, lr in ((1, 1e-3), (2, 5e-4), (3, 2e-3)):
        g = (rng.normal(size=p.size) * 10.0 ** rng.uniform(-4, 0, size=p.size)).astype(np.float32)
        mlp.grad.copy_(torch.from_numpy(g))
        G.gm_mlp_adamw(mlp, lr, weight_decay=0.01)
        p, m, v = M.adamw(p, g.astype(np.float64), m, v, step, lr, weight_decay=0.01)
    got = mlp.params.cpu().numpy().astype(np.float64)
    assert np.abs(got - p).max() <= 1e-6, np.abs(got - p).max()
    assert torch.equal(mlp.params_bf16.float().cpu(), torch.from_numpy(M.bf16(got).astype(np.float32)))


def _features_case(b, omega=None):
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    x, mom = G.gm_features(gm, _dev(b, omega=omega))
    x = x.float().cpu().numpy().astype(np.float64)
    mom = mom.cpu().numpy()
    nbad, ntot = 0, 0
    for g in range(b.n):
        d, s = b.image(b.data, g), b.image(b.sigma, g)
        om = None if omega is None else b.image(omega, g)
        rm = O.moments(d, s, om)
        assert np.allclose(mom[g], rm[:8], rtol=1e-9, atol=1e-9), (g, mom[g], rm)
        rx = M.features(rm, d.astype(np.float64), _usable(d, s, om))
        diff = np.abs(x[g] - rx)
        assert np.all(diff <= 2.0 ** -7 * np.abs(rx) + 1e-30), (g, np.argmax(diff - 2.0 ** -7 * np.abs(rx)))
        nbad += int(np.sum(diff > 0))
        ntot += rx.size
    print(f"features: {nbad} of {ntot} values one BF16 step apart", flush=True)
    assert nbad <= 0.01 * ntot


def test_features_sersic64():
    _features_case(oracle_batch("sersic64", 24, seed=0))


def test_features_uneven_sizes():
    _features_case(oracle_batch("uneven", 6, seed=0))


def test_features_masked():
    mixed = oracle_mixed(40, seed=3)
    b = mixed["sersic"]
    _features_case(b, omega=b.omega)


@pytest.mark.parametrize("case", ["sersic64", "uneven", "masked"])
def test_feature_moments_equal_default_guess_moments(case):
    # the learned fit builds its refit start from the moments the feature pass
    # stores, the plain fit's start recomputes them: the same bits either way
    if case == "masked":
        b = oracle_mixed(40, seed=3)["sersic"]
        omega = b.omega
    else:
        b, omega = oracle_batch(case, 12, seed=1), None
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    db = _dev(b, omega=omega)
    m8 = G.gm_features(gm, db)[1].cpu().numpy()        # sky0 F0 xc yc m_g r0 q0 theta0
    m6 = G.gm_default_guess(gm, db)[1].cpu().numpy()   # xc - W/2, yc - H/2, m_g, ln r0, q0, theta0
    w, h = np.asarray(b.w, np.float64), np.asarray(b.h, np.float64)
    assert np.array_equal(m6[:, 0], m8[:, 2] - 0.5 * w)
    assert np.array_equal(m6[:, 1], m8[:, 3] - 0.5 * h)
    assert np.array_equal(m6[:, 2], m8[:, 4])
    assert np.allclose(m6[:, 3], np.log(m8[:, 5]), rtol=1e-15, atol=1e-15)
    assert np.array_equal(m6[:, 4], m8[:, 6])
    assert np.array_equal(m6[:, 5], m8[:, 7])


def test_targets_and_decode_match_oracle():
    b = oracle_batch("sersic64", 32, seed=5)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    db = _dev(b)
    _, mom = G.gm_features(gm, db)
    tg = G.gm_proposal_targets(gm, db, b.truth, mom).cpu().numpy()
    mom_h = mom.cpu().numpy()
    rng = np.random.default_rng(6)
    out = rng.normal(scale=0.8, size=(b.n, 16)).astype(np.float32)
    out[3, 3] = 40.0                       # re far too large: invalid
    out[5, 4] = -9.0                       # n below the bound: invalid
    params, valid = G.gm_proposal_decode(gm, db, torch.from_numpy(out).cuda(), mom)
    params, valid = params.cpu().numpy(), valid.cpu().numpy()
    for g in range(b.n):
        rm = O.moments(b.image(b.data, g), b.image(b.sigma, g))
        rt = M.targets(b.truth[g], rm)
        assert np.allclose(tg[g], rt, rtol=1e-6, atol=1e-6), (g, tg[g], rt)
        rp, rv = M.decode(out[g], rm, int(b.h[g]), int(b.w[g]))
        assert bool(valid[g]) == rv, g
        assert np.allclose(params[g], rp, rtol=1e-9, atol=1e-9), (g, params[g], rp)
    assert not valid[3] and not valid[5]
    assert np.allclose(mom_h[:, 0], [O.moments(b.image(b.data, g), b.image(b.sigma, g))[0] for g in range(b.n)])


def test_synth_noise_matches_philox_reference():
    rng = np.random.default_rng(7)
    h = np.array([20, 64, 7, 33], np.int32)
    w = np.array([30, 64, 5, 33], np.int32)
    off = np.concatenate([[0], np.cumsum(h.astype(np.int64) * w)[:-1]])
    npix = int(off[-1] + h[-1] * w[-1])
    unit = rng.uniform(0.0, 1.0, npix).astype(np.float32)
    snr = rng.uniform(20, 200, 4)
    sky = rng.uniform(0.5, 1.5, 4)
    seed, first, sigma = 0x123456789, 1000, 1.5
    mag = torch.zeros(4, 3, dtype=torch.float64, device="cuda")
    data, sig = G.gm_synth_noise(h, w, off, torch.from_numpy(unit).cuda(), torch.from_numpy(snr).cuda(),
                                 torch.from_numpy(sky).cuda(), sigma, seed, first_index=first, mag_out=mag[:, 1],
                                 mag_stride=3)
    data, sig, mag = data.cpu().numpy(), sig.cpu().numpy(), mag.cpu().numpy()
    assert np.all(sig == np.float32(sigma))
    for g in range(4):
        o, n = int(off[g]), int(h[g] * w[g])
        u = unit[o:o + n].astype(np.float64)
        F = snr[g] * sigma / u.max()
        ref = F * u + sky[g] + sigma * galaxy_normals(seed, first + g, n)
        assert np.allclose(data[o:o + n], ref, rtol=2e-7, atol=2e-6), g
        assert abs(mag[g, 1] - (22.5 - 2.5 * math.log10(F))) < 1e-12
        assert mag[g, 0] == 0 and mag[g, 2] == 0


def _judge(b, gp, gc, gs):
    """Parity of GPU fits with the oracle LM from the oracle's moment guess
    (judge_fit on every galaxy both sides converge)."""
    om = from_spec(b.model)
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, ostart)
    names = S.MODEL_SPECS[b.model]["names"]
    npass, nboth, fails, counts = judge_batch(b, om, names, gp, gc, gs, rp, rc, rs)
    print(f"  parity verdicts {counts}, fails {fails}", flush=True)
    return npass, nboth, rs, rn


def test_fit_learned_falls_back_on_invalid_proposals():
    b = oracle_batch("sersic64", 12, seed=8)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    db = _dev(b)
    flat = np.zeros(M.param_count(), np.float32)
    M.unpack(flat)[-1][1][3] = 1000.0          # ln re output far out: every proposal invalid
    mlp = G.MLP(flat, train=False)
    lp, lc, ln, ls, fb = [t.cpu().numpy() for t in G.gm_fit_learned(gm, db, mlp)]
    start, _ = G.gm_default_guess(gm, db)
    dp, dc, dn, ds = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start)]
    assert np.all(fb == 1)       # every proposal invalid
    assert np.array_equal(lp, dp) and np.array_equal(lc, dc) and np.array_equal(ln, dn) and np.array_equal(ls, ds)


def test_fit_learned_from_untrained_network_matches_oracle():
    b = oracle_batch("sersic64", 24, seed=9)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    mlp = G.MLP(np.zeros(M.param_count(), np.float32), train=False)    # proposal = moments, n = e^0.6
    lp, lc, ln, ls, fb = [t.cpu().numpy() for t in G.gm_fit_learned(gm, _dev(b), mlp)]
    npass, nboth, rs, _ = _judge(b, lp, lc, ls)
    print(f"untrained proposal: fallback {fb.sum()}/{b.n}, parity {npass}/{nboth}", flush=True)
    assert np.all(ls[fb == 0] == 0) and set(np.unique(fb)) <= {0, 1, 2}
    assert nboth >= 0.8 * b.n and npass == nboth


def test_training_reduces_loss_and_iterations():
    print("training set: 32768 forward-model galaxies", flush=True)
    ds = Lrn.make_training_set(32768, seed=1)
    assert torch.isfinite(ds.t).all() and torch.isfinite(ds.x.float()).all()
    mlp = Lrn.new_mlp(0)
    losses = Lrn.train(mlp, ds, epochs=6, batch=1024)
    print(f"epoch losses {[round(v, 4) for v in losses]} (data {ds.seconds:.2f} s)", flush=True)
    assert losses[-1] < 0.5 * losses[0]
    b = oracle_batch("sersic64", 48, seed=2)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    db = _dev(b)
    lp, lc, ln, ls, fb = [t.cpu().numpy() for t in G.gm_fit_learned(gm, db, mlp)]
    start, _ = G.gm_default_guess(gm, db)
    dp, dc, dn, ds_ = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start)]
    npass, nboth, rs, rn = _judge(b, lp, lc, ls)
    print(f"held-out: iterations learned {ln.mean():.2f} (fallback {fb.sum()}) vs default {dn.mean():.2f} "
          f"(oracle {rn.mean():.2f}); converged learned {np.mean(ls == 0):.3f} default {np.mean(ds_ == 0):.3f}; "
          f"parity {npass}/{nboth}", flush=True)
    assert ln.mean() < dn.mean()
    assert nboth >= 0.8 * b.n and npass == nboth


def test_proposal_trial_budget():
    """With a budget of 2 trials from the learned start, slower fits go to the
    fallback: their result is the moment-start fit and the trials add up."""
    b = oracle_batch("sersic64", 24, seed=10)
    gm = G.Model.from_spec(S.MODEL_SPECS["sersic"])
    db = _dev(b)
    mlp = G.MLP(np.zeros(M.param_count(), np.float32), train=False)
    lp, lc, ln, ls, fb = [t.cpu().numpy() for t in G.gm_fit_learned(gm, db, mlp, proposal_max_iter=2)]
    start, _ = G.gm_default_guess(gm, db)
    dp, dc, dn, ds = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start)]
    sel = fb == 2
    print(f"budget 2: {int(sel.sum())} of {b.n} refitted", flush=True)
    assert sel.sum() >= b.n // 2
    assert np.array_equal(lp[sel], dp[sel]) and np.array_equal(ls[sel], ds[sel])
    assert np.array_equal(ln[sel], dn[sel] + 2)
    assert np.all(ls[fb == 0] == 0) and np.all(ln[fb == 0] <= 2)
