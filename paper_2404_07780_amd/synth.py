"""Seeded synthetic inputs for galaxy-profile fitting.

This module draws what a survey would hand to the fitter -- cutout sizes,
true profile parameters, PSF kernels, sky levels, noise -- and turns a
noiseless *unit-flux* model image into data and sigma images.  It holds none
of the fitting method's arithmetic: the galaxy model image itself is rendered
by whichever side needs it (the HIP library for the benchmark, the FP64
oracle for parity tests), and only its linear scaling to the drawn
signal-to-noise, sky and noise happens here.

Random streams: galaxy ``i`` of configuration ``cfg`` with seed ``seed`` draws
its parameters from ``PCG64(SeedSequence([seed, cfg, i, 0]))`` and its noise
from ``PCG64(SeedSequence([seed, cfg, i, 1]))``, so any subset regenerates
independently of batching.

Workloads (the distributions the fitter is benchmarked on):
  * ``sersic64``  -- 64x64 cutouts, single Sersic + flat sky, Gaussian PSF of
    FWHM 1.5 px on 15x15 (pixel-integrated), sigma = 1, Gaussian noise;
  * ``uneven``    -- square cutouts log-uniform in [48, 256] px, a circular
    Moffat PSF per galaxy (beta 2.5-4.5, FWHM 1.2-2.5 px, 25x25), Poisson
    plus 5 e- read noise;
  * ``bulgedisk`` -- 128x128, Sersic bulge + exponential disk with a shared
    centre, PSF and noise as ``uneven``;
  * ``paper``     -- the shapes of the paper's SDSS test (Sec. 3): 128x128
    single Sersic + sky, one circular Moffat PSF of beta 3 and FWHM 3.03 px
    (1.2 arcsec at 0.396 arcsec/px) on 41x41, noise as ``uneven``; synthetic
    galaxies of the common draw (no survey item is reproduced).
Common Sersic draw: centre (W/2, H/2) + U(-2, 2) px, r_e log-uniform
[2, 15] px, n U(0.5, 6), q U(0.3, 1), PA U(0, 180) deg, peak SNR
log-uniform [20, 200] (peak of the noiseless convolved galaxy without sky
over the noise sigma at that pixel).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from scipy.special import erf

M0 = 22.5
READ_NOISE = 5.0

# profile type codes shared by the C interfaces of both implementations
SERSIC, EXPDISK, FERRER, KING, GAUSSIAN, MOFFAT, SKY, SKYPLANE = range(1, 9)

# Model layouts: list of (type, convolve, idx per natural slot, fixed values).
# Parameter vector of "sersic": x0 y0 mag re n q pa sky.
# Parameter vector of "bulgedisk": x0 y0 | mag_b re_b n_b q_b pa_b | mag_d rs_d q_d pa_d | sky.
MODEL_SPECS: Dict[str, dict] = {
    "sersic": dict(
        p=8,
        comps=[
            (SERSIC, 1, [0, 1, 2, 3, 4, 5, 6], []),
            (SKY, 0, [7], []),
        ],
        names=["x0", "y0", "mag", "re", "n", "q", "pa", "sky"],
    ),
    # single boxy Sersic (B of eq. (r) free) + sky: x0 y0 mag re n q pa box sky
    "sersic_box": dict(
        p=9,
        comps=[
            (SERSIC, 1, [0, 1, 2, 3, 4, 5, 6, 7], []),
            (SKY, 0, [8], []),
        ],
        names=["x0", "y0", "mag", "re", "n", "q", "pa", "box", "sky"],
    ),
    # single King with alpha free (Sec. 4.2.3) + sky: x0 y0 I0 rc rt q pa alpha sky
    "king_free": dict(
        p=9,
        comps=[
            (KING, 1, [0, 1, 2, 3, 4, 5, 6, 7], []),
            (SKY, 0, [8], []),
        ],
        names=["x0", "y0", "I0", "rc", "rt", "q", "pa", "alpha", "sky"],
    ),
    # single Ferrer with a and b free (Sec. 4.2.2) + sky: x0 y0 mag rout q pa a b sky
    "ferrer_free": dict(
        p=9,
        comps=[
            (FERRER, 1, [0, 1, 2, 3, 4, 5, 6, 7], []),
            (SKY, 0, [8], []),
        ],
        names=["x0", "y0", "mag", "rout", "q", "pa", "a", "b", "sky"],
    ),
    # single Sersic + the tilted-plane sky of Appendix D: ... sky kx ky
    "sersic_tilt": dict(
        p=10,
        comps=[
            (SERSIC, 1, [0, 1, 2, 3, 4, 5, 6], []),
            (SKYPLANE, 0, [7, 8, 9], []),
        ],
        names=["x0", "y0", "mag", "re", "n", "q", "pa", "sky", "kx", "ky"],
    ),
    "bulgedisk": dict(
        p=12,
        comps=[
            (SERSIC, 1, [0, 1, 2, 3, 4, 5, 6], []),
            (EXPDISK, 1, [0, 1, 7, 8, 9, 10], []),
            (SKY, 0, [11], []),
        ],
        names=["x0", "y0", "mag_b", "re_b", "n_b", "q_b", "pa_b", "mag_d", "rs_d", "q_d", "pa_d", "sky"],
    ),
    # Sersic + modified Ferrer bar (a = 0.5, b = 1.9 fixed), shared centre
    "sersicbar": dict(
        p=12,
        comps=[
            (SERSIC, 1, [0, 1, 2, 3, 4, 5, 6], []),
            (FERRER, 1, [0, 1, 7, 8, 9, 10, -1, -1], [0, 0, 0, 0, 0, 0, 0.5, 1.9]),
            (SKY, 0, [11], []),
        ],
        names=["x0", "y0", "mag", "re", "n", "q", "pa", "mag_bar", "rout", "q_bar", "pa_bar", "sky"],
    ),
    # circular King cluster (alpha = 2, q = 1, PA = 0 fixed)
    "king": dict(
        p=6,
        comps=[
            (KING, 1, [0, 1, 2, 3, 4, -1, -1, -1], [0, 0, 0, 0, 0, 1.0, 0.0, 2.0]),
            (SKY, 0, [5], []),
        ],
        names=["x0", "y0", "I0", "rc", "rt", "sky"],
    ),
    # unconvolved circular Moffat point source (beta = 3, q = 1, PA = 0 fixed)
    "point": dict(
        p=5,
        comps=[
            (MOFFAT, 0, [0, 1, 2, 3, -1, -1, -1], [0, 0, 0, 0, 1.0, 0.0, 3.0]),
            (SKY, 0, [4], []),
        ],
        names=["x0", "y0", "mag", "fwhm", "sky"],
    ),
}

# columns that carry a component's flux: ("mag", col) shift by -2.5 log10 F,
# ("amp", col) scale by F
FLUX_COLUMNS = {
    "sersic": [("mag", 2)],
    "sersic_tilt": [("mag", 2)],
    "sersic_box": [("mag", 2)],
    "king_free": [("amp", 2)],
    "ferrer_free": [("mag", 2)],
    "bulgedisk": [("mag", 2), ("mag", 7)],
    "sersicbar": [("mag", 2), ("mag", 7)],
    "king": [("amp", 2)],
    "point": [("mag", 2)],
}

CONFIG_IDS = {"sersic64": 1, "uneven": 2, "bulgedisk": 3, "mixed": 5, "paper": 6}


def _rng(seed: int, cfg: int, i: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, cfg, i, stream])))


def gaussian_psf(fwhm: float, k: int) -> np.ndarray:
    """Circular Gaussian kernel integrated over each pixel (erf), sum 1."""
    s = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    c = (k - 1) / 2.0
    e = np.arange(k + 1, dtype=np.float64) - c - 0.5
    cdf = 0.5 * (1.0 + erf(e / (math.sqrt(2.0) * s)))
    p1 = np.diff(cdf)
    ker = np.outer(p1, p1)
    return (ker / ker.sum()).astype(np.float32)


def moffat_psf(beta: float, fwhm: float, k: int, sub: int = 10) -> np.ndarray:
    """Circular Moffat kernel, each pixel the mean of sub x sub samples, sum 1."""
    rd = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
    c = (k - 1) / 2.0
    off = (np.arange(sub) + 0.5) / sub - 0.5
    ax = (np.arange(k)[:, None] - c + off[None, :]).reshape(-1)
    r2 = ax[:, None] ** 2 + ax[None, :] ** 2
    v = (1.0 + r2 / (rd * rd)) ** (-beta)
    ker = v.reshape(k, sub, k, sub).mean(axis=(1, 3))
    return (ker / ker.sum()).astype(np.float32)


@dataclass
class Batch:
    """A ragged batch: concatenated row-major cutouts and PSFs."""

    config: str
    model: str
    h: np.ndarray            # int32 [n]
    w: np.ndarray            # int32 [n]
    img_off: np.ndarray      # int64 [n] offsets into the pixel arrays
    psf_k: np.ndarray        # int32 [n]
    psf_off: np.ndarray      # int64 [n]
    psf: np.ndarray          # float32, concatenated K*K kernels
    truth: np.ndarray        # float64 [n, p]; magnitudes filled by finish()
    snr: np.ndarray          # float64 [n]
    sky: np.ndarray          # float64 [n]
    index: np.ndarray        # int64 [n] galaxy indices within the configuration
    seed: int = 0
    data: Optional[np.ndarray] = None    # float32, filled by finish()
    sigma: Optional[np.ndarray] = None
    omega: Optional[np.ndarray] = None   # uint8 mask (1 = use), or None

    @property
    def n(self) -> int:
        return len(self.h)

    @property
    def npix(self) -> int:
        return int(self.img_off[-1] + self.h[-1].astype(np.int64) * self.w[-1]) if self.n else 0

    def image(self, arr: np.ndarray, g: int) -> np.ndarray:
        o = int(self.img_off[g])
        return arr[o:o + int(self.h[g]) * int(self.w[g])].reshape(int(self.h[g]), int(self.w[g]))

    def psf_of(self, g: int) -> np.ndarray:
        k = int(self.psf_k[g])
        o = int(self.psf_off[g])
        return self.psf[o:o + k * k].reshape(k, k)

    def subset(self, sel) -> "Batch":
        """A new batch holding galaxies `sel` (data copied if present)."""
        sel = np.asarray(sel, dtype=np.int64)
        h, w, k = self.h[sel], self.w[sel], self.psf_k[sel]
        img_off = np.concatenate([[0], np.cumsum(h.astype(np.int64) * w)[:-1]]).astype(np.int64)
        psf_off = np.concatenate([[0], np.cumsum(k.astype(np.int64) * k)[:-1]]).astype(np.int64)
        psf = np.concatenate([self.psf_of(int(g)).ravel() for g in sel]) if len(sel) else np.zeros(0, np.float32)
        out = Batch(self.config, self.model, h.copy(), w.copy(), img_off, k.copy(), psf_off, psf,
                    self.truth[sel].copy(), self.snr[sel].copy(), self.sky[sel].copy(), self.index[sel].copy(),
                    self.seed)
        if self.data is not None:
            out.data = np.concatenate([self.image(self.data, int(g)).ravel() for g in sel])
            out.sigma = np.concatenate([self.image(self.sigma, int(g)).ravel() for g in sel])
        if self.omega is not None:
            out.omega = np.concatenate([self.image(self.omega, int(g)).ravel() for g in sel])
        return out


def _sersic_draw(r: np.random.Generator, h: int, w: int):
    x0 = w / 2.0 + r.uniform(-2.0, 2.0)
    y0 = h / 2.0 + r.uniform(-2.0, 2.0)
    re = math.exp(r.uniform(math.log(2.0), math.log(15.0)))
    n = r.uniform(0.5, 6.0)
    q = r.uniform(0.3, 1.0)
    pa = r.uniform(0.0, 180.0)
    snr = math.exp(r.uniform(math.log(20.0), math.log(200.0)))
    return x0, y0, re, n, q, pa, snr


def free_shape_variant(b: Batch, kind: str) -> Batch:
    """Turn a drawn single-Sersic batch into single King ("king_free") or
    Ferrer ("ferrer_free") galaxies with the same centres, axis ratios,
    angles, SNRs and skies: King r_c = r_e / 2, r_t = U(6, 16) r_c, alpha
    U(1.5, 3), unit amplitude; Ferrer r_out = 2 r_e, a U(1, 3), b U(0, 1.5),
    unit flux.  Extra draws from the galaxy's own generator, stream 2."""
    cfg = CONFIG_IDS[b.config]
    t = np.zeros((b.n, 9))
    for g in range(b.n):
        r = _rng(b.seed, cfg, int(b.index[g]), 2)
        x0, y0, _m, re, _n, q, pa, sky = b.truth[g]
        if kind == "king_free":
            rc = 0.5 * re
            t[g] = [x0, y0, 1.0, rc, r.uniform(6.0, 16.0) * rc, q, pa, r.uniform(1.5, 3.0), sky]
        else:
            t[g] = [x0, y0, M0, 2.0 * re, q, pa, r.uniform(1.0, 3.0), r.uniform(0.0, 1.5), sky]
    b.truth = t
    b.model = kind
    return b


def draw(config: str, n: int, seed: int = 0, start: int = 0) -> Batch:
    """Draw galaxies start..start+n-1 of a workload (no images yet)."""
    cfg = CONFIG_IDS[config]
    hs, ws, ks, psfs, truths, snrs, skies = [], [], [], [], [], [], []
    model = "bulgedisk" if config == "bulgedisk" else "sersic"
    p = MODEL_SPECS[model]["p"]
    gpsf = gaussian_psf(1.5, 15) if config == "sersic64" else None
    ppsf = moffat_psf(3.0, 3.03, 41) if config == "paper" else None
    for i in range(start, start + n):
        r = _rng(seed, cfg, i, 0)
        t = np.zeros(p)
        if config == "sersic64":
            h = w = 64
            x0, y0, re, nn, q, pa, snr = _sersic_draw(r, h, w)
            sky = r.uniform(0.5, 1.5)
            psf = gpsf
            t[:] = [x0, y0, M0, re, nn, q, pa, sky]
        elif config == "uneven":
            side = int(round(math.exp(r.uniform(math.log(48.0), math.log(256.0)))))
            h = w = side
            x0, y0, re, nn, q, pa, snr = _sersic_draw(r, h, w)
            beta = r.uniform(2.5, 4.5)
            fwhm = r.uniform(1.2, 2.5)
            sky = r.uniform(50.0, 200.0)
            psf = moffat_psf(beta, fwhm, 25)
            t[:] = [x0, y0, M0, re, nn, q, pa, sky]
        elif config == "paper":
            h = w = 128
            x0, y0, re, nn, q, pa, snr = _sersic_draw(r, h, w)
            sky = r.uniform(50.0, 200.0)
            psf = ppsf
            t[:] = [x0, y0, M0, re, nn, q, pa, sky]
        elif config == "bulgedisk":
            h = w = 128
            x0 = w / 2.0 + r.uniform(-2.0, 2.0)
            y0 = h / 2.0 + r.uniform(-2.0, 2.0)
            n_b = r.uniform(2.0, 6.0)
            re_b = math.exp(r.uniform(math.log(1.0), math.log(6.0)))
            q_b = r.uniform(0.5, 1.0)
            pa_b = r.uniform(0.0, 180.0)
            re_d = math.exp(r.uniform(math.log(5.0), math.log(25.0)))
            q_d = r.uniform(0.2, 1.0)
            pa_d = r.uniform(0.0, 180.0)
            bt = r.uniform(0.1, 0.9)
            snr = math.exp(r.uniform(math.log(20.0), math.log(200.0)))
            beta = r.uniform(2.5, 4.5)
            fwhm = r.uniform(1.2, 2.5)
            sky = r.uniform(50.0, 200.0)
            psf = moffat_psf(beta, fwhm, 25)
            # magnitudes encode the bulge-to-total split of a unit total flux
            m_b = M0 - 2.5 * math.log10(bt)
            m_d = M0 - 2.5 * math.log10(1.0 - bt)
            t[:] = [x0, y0, m_b, re_b, n_b, q_b, pa_b, m_d, re_d / 1.678346990016661, q_d, pa_d, sky]
        else:
            raise ValueError(config)
        hs.append(h)
        ws.append(w)
        ks.append(psf.shape[0])
        psfs.append(psf.ravel())
        truths.append(t)
        snrs.append(snr)
        skies.append(sky)
    h = np.array(hs, np.int32)
    w = np.array(ws, np.int32)
    k = np.array(ks, np.int32)
    img_off = np.concatenate([[0], np.cumsum(h.astype(np.int64) * w)[:-1]]).astype(np.int64)
    psf_off = np.concatenate([[0], np.cumsum(k.astype(np.int64) * k)[:-1]]).astype(np.int64)
    return Batch(config, model, h, w, img_off, k, psf_off, np.concatenate(psfs).astype(np.float32),
                 np.array(truths), np.array(snrs), np.array(skies), np.arange(start, start + n, dtype=np.int64),
                 seed)


def unit_truth(b: Batch) -> np.ndarray:
    """Parameters to render for finish(): total flux 1 (m = M0 split by the
    drawn bulge fraction for two-component models) and zero sky."""
    t = b.truth.copy()
    spec = MODEL_SPECS[b.model]
    for typ, _conv, idx, _fx in spec["comps"]:
        if typ == SKY:
            t[:, idx[0]] = 0.0
    return t


def finish(b: Batch, unit_images: np.ndarray) -> Batch:
    """Scale unit-flux noiseless renders to the drawn peak SNR, add sky and
    noise.  unit_images: concatenated float64/float32 pixels of the model
    rendered at unit_truth(b).  Fills b.data, b.sigma and the flux columns of
    b.truth (magnitudes shifted, amplitudes scaled)."""
    cfg = CONFIG_IDS[b.config]
    data = np.empty(b.npix, np.float32)
    sigma = np.empty(b.npix, np.float32)
    for g in range(b.n):
        u = np.asarray(b.image(unit_images, g), np.float64)
        peak = float(u.max())
        if not peak > 0.0:
            raise ValueError(f"galaxy {g}: non-positive unit render")
        snr, sky = float(b.snr[g]), float(b.sky[g])
        r = _rng(b.seed, cfg, int(b.index[g]), 1)
        if b.config == "sersic64":
            F = snr * 1.0 / peak
            m_true = F * u + sky
            d = m_true + r.standard_normal(u.shape)
            s = np.ones_like(u)
        else:
            var0 = sky + READ_NOISE ** 2
            P = 0.5 * (snr * snr + math.sqrt(snr ** 4 + 4.0 * snr * snr * var0))
            F = P / peak
            m_true = F * u + sky
            d = r.poisson(m_true).astype(np.float64) + r.normal(0.0, READ_NOISE, u.shape)
            s = np.sqrt(m_true + READ_NOISE ** 2)
        o = int(b.img_off[g])
        npx = u.size
        data[o:o + npx] = d.ravel()
        sigma[o:o + npx] = s.ravel()
        for kind, c in FLUX_COLUMNS[b.model]:
            if kind == "mag":
                b.truth[g, c] = b.truth[g, c] - 2.5 * math.log10(F)
            else:
                b.truth[g, c] = b.truth[g, c] * F
    b.data = data
    b.sigma = sigma
    return b


def _blob_mask(r: np.random.Generator, h: int, w: int, x0: float, y0: float, frac: float = 0.05) -> np.ndarray:
    """Elliptical blobs (semi-major U(2, 8) px, q U(0.3, 1), random PA, centres
    at least 5 px from (x0, y0)) added until at least `frac` of the pixels are
    masked; returns the mask (1 = use)."""
    xx = np.arange(w)[None, :] + 0.5
    yy = h - np.arange(h)[:, None] - 0.5
    m = np.ones((h, w), np.uint8)
    for _ in range(1000):
        if 1.0 - m.mean() >= frac:
            break
        a = r.uniform(2.0, 8.0)
        q = r.uniform(0.3, 1.0)
        th = math.radians(r.uniform(0.0, 180.0))
        cx, cy = r.uniform(0.0, w), r.uniform(0.0, h)
        if math.hypot(cx - x0, cy - y0) < 5.0:
            continue
        dx, dy = xx - cx, yy - cy
        X = math.cos(th) * dx + math.sin(th) * dy
        Y = -math.sin(th) * dx + math.cos(th) * dy
        m[(X / a) ** 2 + (Y / (q * a)) ** 2 <= 1.0] = 0
    return m


MIXED_KINDS = ("sersic", "sersicbar", "king", "point")


def draw_mixed(n: int, seed: int = 0, start: int = 0) -> Dict[str, Batch]:
    """Mixed-profile workload, galaxies start..start+n-1: square cutouts
    log-uniform in [64, 192] px; 60% single Sersic, 20% Sersic + Ferrer bar
    (r_out U(5, 20) px, q U(0.2, 0.5), PA U(0, 180), bar flux fraction
    U(0.1, 0.3)), 10% King (r_c U(1, 5) px, r_t U(10, 60) px with r_t >= 2 r_c),
    10% unconvolved Moffat point source (FWHM that of the galaxy's PSF); a
    25x25 Moffat PSF per galaxy and Poisson + read noise as in "uneven"; at
    least 5% of the pixels masked in elliptical blobs.  Returns one batch per
    model (keys of MIXED_KINDS present)."""
    cfg = CONFIG_IDS["mixed"]
    rows = {k: [] for k in MIXED_KINDS}
    for i in range(start, start + n):
        r = _rng(seed, cfg, i, 0)
        side = int(round(math.exp(r.uniform(math.log(64.0), math.log(192.0)))))
        h = w = side
        u = r.uniform()
        kind = "sersic" if u < 0.6 else "sersicbar" if u < 0.8 else "king" if u < 0.9 else "point"
        beta = r.uniform(2.5, 4.5)
        fwhm = r.uniform(1.2, 2.5)
        psf = moffat_psf(beta, fwhm, 25)
        sky = r.uniform(50.0, 200.0)
        if kind == "sersic":
            x0, y0, re, nn, q, pa, snr = _sersic_draw(r, h, w)
            t = [x0, y0, M0, re, nn, q, pa, sky]
        elif kind == "sersicbar":
            x0, y0, re, nn, q, pa, snr = _sersic_draw(r, h, w)
            rout = r.uniform(5.0, 20.0)
            qb = r.uniform(0.2, 0.5)
            pab = r.uniform(0.0, 180.0)
            fb = r.uniform(0.1, 0.3)
            t = [x0, y0, M0 - 2.5 * math.log10(1.0 - fb), re, nn, q, pa, M0 - 2.5 * math.log10(fb), rout, qb, pab,
                 sky]
        elif kind == "king":
            x0 = w / 2.0 + r.uniform(-2.0, 2.0)
            y0 = h / 2.0 + r.uniform(-2.0, 2.0)
            rc = r.uniform(1.0, 5.0)
            rt = max(r.uniform(10.0, 60.0), 2.0 * rc)
            snr = math.exp(r.uniform(math.log(20.0), math.log(200.0)))
            t = [x0, y0, 1.0, rc, rt, sky]
        else:
            x0 = w / 2.0 + r.uniform(-2.0, 2.0)
            y0 = h / 2.0 + r.uniform(-2.0, 2.0)
            snr = math.exp(r.uniform(math.log(20.0), math.log(200.0)))
            t = [x0, y0, M0, fwhm, sky]
        mask = _blob_mask(r, h, w, x0, y0)
        rows[kind].append((i, h, w, psf, np.array(t), snr, sky, mask))
    out = {}
    for kind, lst in rows.items():
        if not lst:
            continue
        h = np.array([x[1] for x in lst], np.int32)
        w = np.array([x[2] for x in lst], np.int32)
        k = np.full(len(lst), 25, np.int32)
        img_off = np.concatenate([[0], np.cumsum(h.astype(np.int64) * w)[:-1]]).astype(np.int64)
        psf_off = np.arange(len(lst), dtype=np.int64) * 625
        b = Batch("mixed", kind, h, w, img_off, k, psf_off, np.concatenate([x[3].ravel() for x in lst]),
                  np.array([x[4] for x in lst]), np.array([x[5] for x in lst]), np.array([x[6] for x in lst]),
                  np.array([x[0] for x in lst], np.int64), seed)
        b.omega = np.concatenate([x[7].ravel() for x in lst])
        out[kind] = b
    return out
