"""FP64 oracle of the learned proposal: cutout features, target encoding and
decoding, the MLP forward and backward passes, and the AdamW update.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): the test suite, the
smoke check and the CPU-baseline leg of the benchmark may use it; the product
package never imports it.  Plain numpy in float64.

The paper motivates a learned initial guess by the deep-learning parameter
estimators it surveys (Sec. 1) and by its own limitation that initial
parameters have to be chosen by hand (Sec. 7); it fixes no network.  What is
computed here is this project's design, stated once:

Features (1056 values per galaxy).  With the image moments of the default
guess (sky0, F0, centroid, m_g, r0, q0, th0) and F0' = max(F0, 1):
  * 32x32 area-weighted cells: cell (a, b) covers rows [a H/32, (a+1) H/32)
    and columns [b W/32, (b+1) W/32) of the pixel grid; its value is the mean
    of D - sky0 over the usable part of its area, times the cell area
    H W / 1024, and the feature is 32 * value / F0' (0 for a cell with no
    usable area);
  * 6 moment features: (xc - W/2)/2, (yc - H/2)/2, (m_g - 14)/2, ln r0 - 1.5,
    e0 cos 2 th0, e0 sin 2 th0 with e0 = (1 - q0)/(1 + q0);
  * 26 zeros (the width is a multiple of 32).
Targets (7 used of 16 outputs), from a single-Sersic truth with q <= 1:
  x0 - xc, y0 - yc, (m - m_g)/0.5, (ln re - 1.7)/0.6, (ln n - 0.6)/0.6,
  e cos 2 theta / 0.3, e sin 2 theta / 0.3 with e = (1 - q)/(1 + q).
Decoding inverts the targets; the ellipticity is capped at 0.9 (q >= 1/19)
and the sky start is sky0.  A proposal is valid when it is finite and inside
the LM bounds.

Network: Linear(1056, 512) -> GELU -> Linear(512, 512) -> GELU ->
Linear(512, 512) -> GELU -> Linear(512, 16), GELU the exact erf form.  FP32
master weights; the products use BF16 copies of the weights, the BF16 input
features, BF16 hidden activations and BF16 backward signals, each rounded to
nearest even from the value the layer produced; sums are exact here (float64)
and FP32 on the device.  Loss: mean over the batch and the 7 used outputs of
the squared error.
"""
from __future__ import annotations

import math

import numpy as np

IN_DIM, HIDDEN, N_HIDDEN, OUT_DIM, N_OUT = 1056, 512, 3, 16, 7
CELLS = 32
X_SCALE = 32.0
# target standardisation: (offset, scale) per output; outputs 0, 1 are raw px
T_MAG_SCALE = 0.5
T_LNRE = (1.7, 0.6)
T_LNN = (0.6, 0.6)
T_E_SCALE = 0.3
E_CAP = 0.9


# ---------------------------------------------------------------- BF16 ---
def bf16(x):
    """Round to the nearest BF16 value (ties to even) through FP32, as float64.
    NaN stays NaN; overflow goes to +-inf like the hardware conversion."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def _ident(x):
    return np.asarray(x, dtype=np.float64)


# ---------------------------------------------------------------- GELU ---
_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    """z * Phi(z) with Phi the standard normal CDF (erf form)."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


# ------------------------------------------------------------ layout -----
def layer_dims(in_dim=IN_DIM, hidden=HIDDEN, n_hidden=N_HIDDEN, out_dim=OUT_DIM):
    dims = [in_dim] + [hidden] * n_hidden + [out_dim]
    return [(dims[l], dims[l + 1]) for l in range(len(dims) - 1)]


def param_count(in_dim=IN_DIM, hidden=HIDDEN, n_hidden=N_HIDDEN, out_dim=OUT_DIM):
    return sum(o * i + o for i, o in layer_dims(in_dim, hidden, n_hidden, out_dim))


def unpack(flat, in_dim=IN_DIM, hidden=HIDDEN, n_hidden=N_HIDDEN, out_dim=OUT_DIM):
    """Flat parameter vector -> [(W [out][in], b [out]), ...] (views)."""
    out, off = [], 0
    for i, o in layer_dims(in_dim, hidden, n_hidden, out_dim):
        W = flat[off: off + o * i].reshape(o, i)
        off += o * i
        b = flat[off: off + o]
        off += o
        out.append((W, b))
    return out


def init_params(seed: int, in_dim=IN_DIM, hidden=HIDDEN, n_hidden=N_HIDDEN, out_dim=OUT_DIM, n_out=N_OUT):
    """Weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)) as FP32, biases 0; the output
    rows past the n_out used outputs are 0."""
    rng = np.random.default_rng(seed)
    flat = np.zeros(param_count(in_dim, hidden, n_hidden, out_dim), np.float32)
    layers = unpack(flat, in_dim, hidden, n_hidden, out_dim)
    for l, (W, b) in enumerate(layers):
        lim = 1.0 / math.sqrt(W.shape[1])
        W[...] = rng.uniform(-lim, lim, size=W.shape).astype(np.float32)
        if l == len(layers) - 1:
            W[n_out:] = 0.0
    return flat


# ----------------------------------------------------------- network -----
def forward(flat, x, emulate_bf16: bool = True, dims=None):
    """x [B][in] (values already BF16 when emulating) -> (out [B][out_dim],
    cache for backward)."""
    rnd = bf16 if emulate_bf16 else _ident
    layers = unpack(np.asarray(flat, np.float64), *(dims or ()))
    a = np.asarray(x, np.float64)
    acts, zs = [a], []
    for l, (W, b) in enumerate(layers):
        z = a @ rnd(W).T + b
        if l < len(layers) - 1:
            zs.append(z)
            a = rnd(gelu(z))
            acts.append(a)
        else:
            out = z
    return out, (acts, zs)


def loss_and_grad(flat, x, targets, emulate_bf16: bool = True, n_out: int = N_OUT, dims=None):
    """MSE over the batch and the first n_out outputs; returns (loss, flat
    gradient, outputs)."""
    rnd = bf16 if emulate_bf16 else _ident
    flat = np.asarray(flat, np.float64)
    out, (acts, zs) = forward(flat, x, emulate_bf16, dims)
    B = out.shape[0]
    t = np.asarray(targets, np.float64)
    diff = np.zeros_like(out)
    diff[:, :n_out] = out[:, :n_out] - t[:, :n_out]
    loss = float(np.sum(diff * diff) / (B * n_out))
    layers = unpack(flat, *(dims or ()))
    grad = np.zeros_like(flat)
    glayers = unpack(grad, *(dims or ()))
    dz = rnd(2.0 * diff / (B * n_out))
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        gW, gb = glayers[l]
        gW[...] = dz.T @ acts[l]
        gb[...] = dz.sum(axis=0)
        if l > 0:
            da = dz @ rnd(W)
            dz = rnd(da * gelu_grad(zs[l - 1]))
    return loss, grad, out


def adamw(flat, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One decoupled-weight-decay Adam step (Loshchilov and Hutter); step
    counts from 1.  Returns new (params, m, v)."""
    p = np.asarray(flat, np.float64) * (1.0 - lr * weight_decay)
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


# ---------------------------------------------------------- features -----
def _overlap(lo, hi, n_pix):
    """Length of [i, i+1) n [lo, hi) for every pixel index i."""
    i = np.arange(n_pix, dtype=np.float64)
    return np.clip(np.minimum(i + 1.0, hi) - np.maximum(i, lo), 0.0, None)


def cell_flux(data, usable, sky0):
    """32x32 area-weighted cells of one cutout: mean of D - sky0 over the usable
    part of each cell times the cell area (0 where nothing is usable)."""
    H, W = data.shape
    dp = np.where(usable, data.astype(np.float64) - sky0, 0.0)
    u = usable.astype(np.float64)
    area = H * W / float(CELLS * CELLS)
    c = np.zeros((CELLS, CELLS))
    for a in range(CELLS):
        orow = _overlap(a * H / CELLS, (a + 1) * H / CELLS, H)
        for b in range(CELLS):
            ocol = _overlap(b * W / CELLS, (b + 1) * W / CELLS, W)
            wgt = np.outer(orow, ocol)
            den = np.sum(wgt * u)
            if den > 0.0:
                c[a, b] = np.sum(wgt * dp) / den * area
    return c


def features(mom, data, usable, rounded: bool = True):
    """One galaxy: mom = oracle moments {sky0, F0, xc, yc, m_g, r0, q0, th0,
    peak}; data [H][W]; usable [H][W] bool.  Returns the 1056 features (BF16
    values as float64 when rounded)."""
    H, W = data.shape
    sky0, F0, xc, yc, mg, r0, q0, th0 = (float(v) for v in mom[:8])
    x = np.zeros(IN_DIM)
    x[:1024] = X_SCALE * cell_flux(data, usable, sky0).ravel() / max(F0, 1.0)
    e0 = (1.0 - q0) / (1.0 + q0)
    x[1024:1030] = [(xc - 0.5 * W) / 2.0, (yc - 0.5 * H) / 2.0, (mg - 14.0) / 2.0, math.log(r0) - 1.5,
                    e0 * math.cos(2.0 * th0), e0 * math.sin(2.0 * th0)]
    return bf16(x) if rounded else x


def targets(truth, mom):
    """Single-Sersic truth (x0, y0, mag, re, n, q, pa[deg], ...) with q <= 1 ->
    the 16 outputs' targets (7 used)."""
    x0, y0, m, re, n, q, pa = (float(v) for v in truth[:7])
    xc, yc, mg = float(mom[2]), float(mom[3]), float(mom[4])
    e = (1.0 - q) / (1.0 + q)
    th = math.radians(pa)
    t = np.zeros(OUT_DIM)
    t[:7] = [x0 - xc, y0 - yc, (m - mg) / T_MAG_SCALE, (math.log(re) - T_LNRE[0]) / T_LNRE[1],
             (math.log(n) - T_LNN[0]) / T_LNN[1], e * math.cos(2.0 * th) / T_E_SCALE,
             e * math.sin(2.0 * th) / T_E_SCALE]
    return t


def decode(out, mom, h: int, w: int):
    """Network outputs -> (x0, y0, mag, re, n, q, pa[deg], sky) and validity
    (finite and inside the LM bounds)."""
    o = [float(v) for v in out[:7]]
    sky0, xc, yc, mg = float(mom[0]), float(mom[2]), float(mom[3]), float(mom[4])
    x0, y0 = xc + o[0], yc + o[1]
    m = mg + T_MAG_SCALE * o[2]
    re = math.exp(T_LNRE[0] + T_LNRE[1] * o[3]) if o[3] < 700 else math.inf
    n = math.exp(T_LNN[0] + T_LNN[1] * o[4]) if o[4] < 700 else math.inf
    e1, e2 = T_E_SCALE * o[5], T_E_SCALE * o[6]
    e = min(math.hypot(e1, e2), E_CAP)
    q = (1.0 - e) / (1.0 + e)
    pa = math.degrees(0.5 * math.atan2(e2, e1))
    if pa < 0.0:
        pa += 180.0
    if pa >= 180.0:
        pa -= 180.0
    p = np.array([x0, y0, m, re, n, q, pa, sky0])
    big = 2.0 * max(h, w)
    valid = bool(np.all(np.isfinite(p)) and 0.0 <= x0 <= w and 0.0 <= y0 <= h and 0.1 <= re <= big
                 and 0.2 <= n <= 10.0)
    return p, valid
