"""Learned proposal: training data made on the device by the forward model,
MLP training through the library's BF16 matrix-core kernels, and the
learned-start fit.

Every step runs in libgmfit's kernels (gm_model_image renders noiseless
unit-flux galaxies, gm_synth_noise scales them to their peak SNR and adds
Philox noise, gm_features / gm_proposal_targets encode them,
gm_mlp_train_step trains); this module draws the truth parameters on the
host, keeps the device tensors and drives the loop.

Training galaxies follow the single-Sersic 64 x 64 workload: centre within
+-2 px of the cutout centre, R_e log-uniform in [2, 15] px, n uniform in
[0.5, 6], q uniform in [0.3, 1], PA uniform in [0, 180) deg, peak SNR
log-uniform in [20, 200] at unit noise sigma, sky uniform in [0.5, 1.5], the
Gaussian PSF of FWHM 1.5 px on 15 x 15 pixels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import gmfit as G
from . import synth as S

IN_DIM, HIDDEN, N_HIDDEN, OUT_DIM, N_OUT = 1056, 512, 3, 16, 7
SIDE = 64


def sersic_model() -> G.Model:
    return G.Model.from_spec(S.MODEL_SPECS["sersic"])


def param_count(in_dim=IN_DIM, hidden=HIDDEN, n_hidden=N_HIDDEN, out_dim=OUT_DIM) -> int:
    dims = [in_dim] + [hidden] * n_hidden + [out_dim]
    return sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1))


def init_params(seed: int, in_dim=IN_DIM, hidden=HIDDEN, n_hidden=N_HIDDEN, out_dim=OUT_DIM,
                n_out=N_OUT) -> np.ndarray:
    """FP32 flat vector: W_l ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), b_l = 0, and
    the rows of the last layer past the n_out used outputs 0."""
    rng = np.random.default_rng(seed)
    dims = [in_dim] + [hidden] * n_hidden + [out_dim]
    parts = []
    for l in range(len(dims) - 1):
        fan_in, fan_out = dims[l], dims[l + 1]
        lim = 1.0 / math.sqrt(fan_in)
        W = rng.uniform(-lim, lim, size=(fan_out, fan_in)).astype(np.float32)
        if l == len(dims) - 2:
            W[n_out:] = 0.0
        parts += [W.ravel(), np.zeros(fan_out, np.float32)]
    return np.concatenate(parts)


def new_mlp(seed: int = 0, device=None, train: bool = True) -> G.MLP:
    return G.MLP(init_params(seed), IN_DIM, HIDDEN, N_HIDDEN, OUT_DIM, N_OUT, device=device, train=train)


def draw_truth(n: int, seed: int) -> dict:
    """Truth parameters of n training galaxies from one generator (vectorised)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 4])))
    return dict(
        x0=SIDE / 2.0 + rng.uniform(-2.0, 2.0, n),
        y0=SIDE / 2.0 + rng.uniform(-2.0, 2.0, n),
        re=np.exp(rng.uniform(math.log(2.0), math.log(15.0), n)),
        n=rng.uniform(0.5, 6.0, n),
        q=rng.uniform(0.3, 1.0, n),
        pa=rng.uniform(0.0, 180.0, n),
        snr=np.exp(rng.uniform(math.log(20.0), math.log(200.0), n)),
        sky=rng.uniform(0.5, 1.5, n),
    )


@dataclass
class DeviceSet:
    x: torch.Tensor          # [n][1056] BF16 features
    t: torch.Tensor          # [n][16] FP32 targets
    seconds: float = 0.0


def _uniform_batch(n: int, data, sigma, psf: np.ndarray, device) -> G.Batch:
    h = np.full(n, SIDE, np.int32)
    off = np.arange(n, dtype=np.int64) * SIDE * SIDE
    k = psf.shape[0]
    return G.Batch(h, h, off, np.full(n, k, np.int32), np.zeros(n, np.int64), data, sigma, psf.ravel(),
                   device=device)


def make_training_set(n: int, seed: int, chunk: int = 65536, device=None,
                      ctx: Optional[G.Context] = None) -> DeviceSet:
    """Features and targets of n forward-model galaxies, built chunk by chunk
    on the device."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ctx = ctx or G.context(dev.index)
    model = sersic_model()
    psf = S.gaussian_psf(1.5, 15).astype(np.float32)
    tr = draw_truth(n, seed)
    X = torch.empty(n, IN_DIM, dtype=torch.bfloat16, device=dev)
    T = torch.empty(n, OUT_DIM, dtype=torch.float32, device=dev)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        m = e - s
        truth = np.stack([tr["x0"][s:e], tr["y0"][s:e], np.full(m, S.M0), tr["re"][s:e], tr["n"][s:e],
                          tr["q"][s:e], tr["pa"][s:e], np.zeros(m)], axis=1)
        truth_d = torch.from_numpy(truth).to(dev)
        unused = torch.empty(m * SIDE * SIDE, device=dev)     # pixels are not read by gm_model_image
        b = _uniform_batch(m, unused, unused, psf, dev)
        unit = G.gm_model_image(model, b, truth_d, ctx=ctx)
        del unused
        snr = torch.from_numpy(np.ascontiguousarray(tr["snr"][s:e])).to(dev)
        sky = torch.from_numpy(np.ascontiguousarray(tr["sky"][s:e])).to(dev)
        data, sig = G.gm_synth_noise(b.h, b.w, b.img_off, unit, snr, sky, 1.0, seed, first_index=s, m0=S.M0,
                                     mag_out=truth_d[:, 2], mag_stride=model.p, ctx=ctx)
        truth_d[:, 7] = sky
        del unit
        b = _uniform_batch(m, data, sig, psf, dev)
        x, mom = G.gm_features(model, b, ctx=ctx)
        X[s:e] = x
        T[s:e] = G.gm_proposal_targets(model, b, truth_d, mom, OUT_DIM, ctx=ctx)
        del data, sig, x, mom, b
    torch.cuda.synchronize(dev)
    return DeviceSet(X, T, time.perf_counter() - t0)


def cosine_lr(step: int, total: int, lr_max: float, lr_min: float) -> float:
    return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * min(step, total) / max(total, 1)))


def train(mlp: G.MLP, ds: DeviceSet, epochs: int, batch: int = 4096, lr_max: float = 1e-3, lr_min: float = 1e-5,
          weight_decay: float = 0.01, seed: int = 0, ctx: Optional[G.Context] = None) -> List[float]:
    """AdamW with a cosine learning rate over shuffled mini-batches; returns
    the mean loss of each epoch."""
    ctx = ctx or G.context(mlp.device.index)
    n = ds.x.shape[0]
    steps = n // batch
    total = steps * epochs
    rng = np.random.default_rng(seed)
    losses = torch.empty(max(total, 1), dtype=torch.float64, device=mlp.device)
    out = []
    k = 0
    for e in range(epochs):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(mlp.device)
        for s in range(steps):
            rows = perm[s * batch:(s + 1) * batch]
            G.gm_mlp_train_step(mlp, ds.x, ds.t, rows, cosine_lr(k, total, lr_max, lr_min),
                                weight_decay=weight_decay, loss=losses[k], ctx=ctx)
            k += 1
        out.append(float(losses[e * steps:(e + 1) * steps].mean().item()))
    return out
