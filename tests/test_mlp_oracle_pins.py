"""Pins of the learned-proposal oracle (oracle/mlp.py) against things other
than itself: torch's own BF16 conversion, its autograd and AdamW, closed forms
of GELU, central finite differences, brute-force block sums and the
partition-of-unity of the area-weighted cells."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import mlp as M

torch = pytest.importorskip("torch")

TINY = (24, 10, 2, 5)          # in, hidden, n_hidden, out


def _tiny(seed=0, n_out=3):
    return M.init_params(seed, *TINY, n_out=n_out).astype(np.float64)


# ------------------------------------------------------------- BF16 -------
def test_bf16_matches_torch_conversion():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, size=4000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40, -1e-42]])
    # exact ties: FP32 values whose low 16 bits are 0x8000
    e = rng.integers(1, 254, size=500, dtype=np.uint32)
    mant = rng.integers(0, 2 ** 7, size=500, dtype=np.uint32)
    ties = (e << 23) | (mant << 16) | np.uint32(0x8000)
    x = np.concatenate([x, ties.view(np.float32).astype(np.float64)])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = M.bf16(x)
    assert np.array_equal(got, ref)


def test_bf16_nan_and_overflow():
    got = M.bf16(np.array([np.nan, np.inf, -np.inf, 3.4e38]))
    assert np.isnan(got[0]) and got[1] == np.inf and got[2] == -np.inf and got[3] == np.inf


# ------------------------------------------------------------- GELU -------
def test_gelu_closed_forms():
    # gelu(z) = z Phi(z); Phi(1) = 0.841344746068543, Phi(-1) = 0.158655253931457
    assert M.gelu(0.0) == 0.0
    assert abs(M.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(M.gelu(-1.0) + 0.15865525393145707) < 1e-15
    z = np.linspace(-6, 6, 101)
    # gelu(z) - gelu(-z) = z (Phi(z) + Phi(-z) = 1)
    assert np.allclose(M.gelu(z) - M.gelu(-z), z, rtol=0, atol=1e-14)
    # gelu'(0) = 1/2; gelu' -> 1 and 0 in the tails
    assert abs(M.gelu_grad(0.0) - 0.5) < 1e-15
    assert abs(M.gelu_grad(8.0) - 1.0) < 1e-12 and abs(M.gelu_grad(-8.0)) < 1e-12


def test_gelu_grad_finite_difference():
    z = np.linspace(-5, 5, 41) + 0.013
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(z), fd, rtol=0, atol=1e-8)


def test_gelu_matches_torch():
    z = torch.linspace(-7, 7, 301, dtype=torch.float64, requires_grad=True)
    y = torch.nn.functional.gelu(z, approximate="none")
    (g,) = torch.autograd.grad(y.sum(), z)
    # absolute floor: 1 + erf(z/sqrt 2) cancels in the negative tail on both sides
    assert np.allclose(M.gelu(z.detach().numpy()), y.detach().numpy(), rtol=1e-14, atol=1e-15)
    assert np.allclose(M.gelu_grad(z.detach().numpy()), g.numpy(), rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------- network ------
def _torch_net(flat, dims):
    layers = M.unpack(np.asarray(flat, np.float64), *dims)
    ts = [(torch.tensor(W.copy(), requires_grad=True), torch.tensor(b.copy(), requires_grad=True))
          for W, b in layers]

    def run(x):
        a = x
        for l, (W, b) in enumerate(ts):
            a = torch.nn.functional.linear(a, W, b)
            if l < len(ts) - 1:
                a = torch.nn.functional.gelu(a, approximate="none")
        return a

    return ts, run


def test_param_layout_and_count():
    assert M.param_count() == 1056 * 512 + 512 + 2 * (512 * 512 + 512) + 16 * 512 + 16
    p = M.init_params(3)
    W_out, b_out = M.unpack(p)[-1]
    assert W_out.shape == (16, 512) and np.all(W_out[7:] == 0) and np.all(b_out == 0)
    W1, _ = M.unpack(p)[0]
    assert np.abs(W1).max() <= 1 / math.sqrt(1056)


def test_exact_forward_matches_torch():
    rng = np.random.default_rng(2)
    flat = _tiny(1) + rng.normal(scale=0.1, size=M.param_count(*TINY))
    x = rng.normal(size=(9, TINY[0]))
    out, _ = M.forward(flat, x, emulate_bf16=False, dims=TINY)
    _, run = _torch_net(flat, TINY)
    ref = run(torch.tensor(x)).detach().numpy()
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-14)


def test_exact_gradient_matches_torch_autograd():
    rng = np.random.default_rng(3)
    flat = _tiny(2) + rng.normal(scale=0.1, size=M.param_count(*TINY))
    x = rng.normal(size=(7, TINY[0]))
    t = rng.normal(size=(7, TINY[3]))
    loss, grad, _ = M.loss_and_grad(flat, x, t, emulate_bf16=False, n_out=3, dims=TINY)
    ts, run = _torch_net(flat, TINY)
    o = run(torch.tensor(x))
    tl = ((o[:, :3] - torch.tensor(t[:, :3])) ** 2).sum() / (7 * 3)
    tl.backward()
    ref = np.concatenate([np.concatenate([W.grad.numpy().ravel(), b.grad.numpy()]) for W, b in ts])
    assert abs(loss - tl.item()) < 1e-14 * max(1.0, abs(loss))
    assert np.allclose(grad, ref, rtol=1e-12, atol=1e-15)


def test_exact_gradient_finite_difference():
    rng = np.random.default_rng(4)
    flat = _tiny(3) + rng.normal(scale=0.2, size=M.param_count(*TINY))
    x = rng.normal(size=(5, TINY[0]))
    t = rng.normal(size=(5, TINY[3]))
    _, grad, _ = M.loss_and_grad(flat, x, t, emulate_bf16=False, n_out=3, dims=TINY)
    h = 1e-6
    for k in rng.choice(len(flat), size=40, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[k] += h
        fm[k] -= h
        lp = M.loss_and_grad(fp, x, t, emulate_bf16=False, n_out=3, dims=TINY)[0]
        lm = M.loss_and_grad(fm, x, t, emulate_bf16=False, n_out=3, dims=TINY)[0]
        assert abs((lp - lm) / (2 * h) - grad[k]) <= 1e-7 * max(1.0, abs(grad[k])), k


def test_unused_outputs_get_no_gradient():
    rng = np.random.default_rng(5)
    flat = M.init_params(0).astype(np.float64)
    x = M.bf16(rng.normal(size=(4, 1056)))
    t = rng.normal(size=(4, 16))
    _, grad, out = M.loss_and_grad(flat, x, t)
    gW, gb = M.unpack(grad)[-1]
    assert np.all(gW[7:] == 0) and np.all(gb[7:] == 0)
    assert np.all(out[:, 7:] == 0)


def test_bf16_forward_within_rounding_of_exact():
    rng = np.random.default_rng(6)
    flat = M.init_params(1).astype(np.float64)
    x = M.bf16(rng.normal(size=(16, 1056)))
    eo, _ = M.forward(flat, x, emulate_bf16=False)
    bo, _ = M.forward(flat, x, emulate_bf16=True)
    # a few BF16 roundings (relative 2^-9 each) per layer
    scale = np.abs(eo[:, :7]).max()
    assert np.abs(bo[:, :7] - eo[:, :7]).max() <= 0.03 * scale
    assert not np.array_equal(bo, eo)


def test_adamw_matches_torch():
    rng = np.random.default_rng(7)
    p0 = rng.normal(size=50)
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 5):
        g = rng.normal(size=50) * 10.0 ** (-step)
        tp.grad = torch.tensor(g.copy())
        opt.step()
        p, m, v = M.adamw(p, g, m, v, step, 3e-3, weight_decay=0.01)
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


# --------------------------------------------------------- features ------
def test_cells_are_block_sums_for_64():
    rng = np.random.default_rng(8)
    d = rng.normal(size=(64, 64)) + 3.0
    c = M.cell_flux(d, np.ones((64, 64), bool), 1.25)
    ref = (d - 1.25).reshape(32, 2, 32, 2).sum(axis=(1, 3))
    assert np.allclose(c, ref, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("h,w", [(48, 80), (37, 37), (192, 100), (20, 31)])
def test_cells_partition_the_flux(h, w):
    rng = np.random.default_rng(h * w)
    d = rng.normal(size=(h, w))
    c = M.cell_flux(d, np.ones((h, w), bool), 0.0)
    assert abs(c.sum() - d.sum()) <= 1e-10 * np.abs(d).sum()


def test_cells_of_constant_image_with_mask():
    rng = np.random.default_rng(9)
    h, w = 50, 70
    usable = rng.uniform(size=(h, w)) > 0.3
    d = np.where(usable, 7.5, 1e6)                  # masked pixels never enter
    c = M.cell_flux(d, usable, 2.5)
    assert np.allclose(c, 5.0 * h * w / 1024, rtol=1e-12)
    none = M.cell_flux(d, np.zeros((h, w), bool), 2.5)
    assert np.all(none == 0)


def test_feature_vector_layout():
    rng = np.random.default_rng(10)
    d = (rng.normal(size=(64, 64)) + 0.8).astype(np.float32)
    d[28:36, 26:40] += 40.0
    s = np.ones_like(d)
    mom = O.moments(d, s)
    x = M.features(mom, d, np.ones(d.shape, bool))
    sky0, F0, xc, yc, mg, r0, q0, th0 = mom[:8]
    assert np.all(x[1030:] == 0)
    assert np.array_equal(x, M.bf16(x))
    blocks = (d.astype(np.float64) - sky0).reshape(32, 2, 32, 2).sum(axis=(1, 3))
    assert np.allclose(x[:1024], M.bf16(32 * blocks.ravel() / F0), rtol=0, atol=0)
    e0 = (1 - q0) / (1 + q0)
    assert np.array_equal(x[1024:1030], M.bf16([(xc - 32) / 2, (yc - 32) / 2, (mg - 14) / 2, math.log(r0) - 1.5,
                                                e0 * math.cos(2 * th0), e0 * math.sin(2 * th0)]))


# ------------------------------------------------- targets / decode ------
def test_decode_inverts_targets():
    rng = np.random.default_rng(11)
    for _ in range(200):
        h = w = int(rng.integers(40, 200))
        truth = [w / 2 + rng.uniform(-2, 2), h / 2 + rng.uniform(-2, 2), rng.uniform(12, 20),
                 math.exp(rng.uniform(math.log(2), math.log(15))), rng.uniform(0.5, 6), rng.uniform(0.3, 1),
                 rng.uniform(0, 180)]
        mom = np.array([rng.uniform(0.5, 1.5), 1e3, w / 2 + rng.normal(), h / 2 + rng.normal(),
                        truth[2] + rng.normal(scale=0.3), 4.0, 0.7, 0.3, 10.0])
        t = M.targets(truth, mom)
        assert np.all(t[7:] == 0)
        p, valid = M.decode(t, mom, h, w)
        assert valid
        assert np.allclose(p[:6], truth[:6], rtol=1e-12, atol=1e-10)
        d = (p[6] - truth[6] + 90) % 180 - 90
        if truth[5] < 1 - 1e-9:
            assert abs(d) < 1e-9
        assert p[7] == mom[0]


def test_decode_caps_ellipticity_and_flags_invalid():
    mom = np.array([1.0, 1e3, 32.0, 32.0, 15.0, 4.0, 0.7, 0.0, 10.0])
    out = np.zeros(16)
    out[5] = 10.0                              # e = 3 -> capped at 0.9
    p, valid = M.decode(out, mom, 64, 64)
    assert valid and abs(p[5] - 0.1 / 1.9) < 1e-15 and p[6] == 0.0
    out[5], out[6] = 0.0, 1.0                  # e2 > 0, e1 = 0: PA 45 deg
    p, _ = M.decode(out, mom, 64, 64)
    assert abs(p[6] - 45.0) < 1e-12
    for k, v in ((0, 40.0), (3, 20.0), (4, -10.0), (4, 10.0), (2, np.nan)):
        o = np.zeros(16)
        o[k] = v
        assert not M.decode(o, mom, 64, 64)[1], (k, v)
