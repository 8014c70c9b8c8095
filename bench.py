"""Benchmark: galaxies fitted per second by batched Levenberg-Marquardt on one
MI355X.

One step = the whole hot path over one batch of synthetic galaxies resident
in HBM: moment-based start vectors (gm_default_guess), the persistent LM fit
(gm_fit_batch) and the covariance errors (gm_param_errors).

Workload "uneven" (default): 8,192 single-Sersic galaxies, square cutouts
log-uniform in 48-256 px, each with its own 25x25 Moffat PSF, Poisson + read
noise.  The images are rendered with the library's own forward model
(gm_model_image) from seeded draws, then noised on the host.

Printed: one JSON line with the throughput, the roofline of the dominant
kernel (the LM fit), and the FP64 CPU oracle timed on a bounded sample of the
same workload; on that sample the oracle also renders the data and the GPU
fit is compared with the oracle fit from the same start (parity).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import torch  # noqa: E402

from paper_2404_07780_amd import gmfit as G  # noqa: E402
from paper_2404_07780_amd import synth as S  # noqa: E402

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak

# HBM bytes per lm_fit launch on the default workload (8192 galaxies, seed 0) from
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0 from a
# 1 GiB copy), keyed by the hash of the kernel sources they were taken with.
TRAFFIC = {"1e071d0ae89bc2a0": 6.485e6 * 1024 * 2.0 + 2.488e4 * 1024}


def kernel_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("gm_abi.hip", "gm_kernels.h", "gm_device.h"):
        with open(os.path.join(ROOT, "paper_2404_07780_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
WORKLOADS = {
    "uneven": dict(n=8192, desc="8192 single-Sersic galaxies, square cutouts log-uniform 48-256 px, per-galaxy "
                                "Moffat PSF 25x25, Poisson + 5 e- read noise, LM from moment-based start"),
    "sersic64": dict(n=64, desc="64 single-Sersic galaxies, 64x64, Gaussian PSF FWHM 1.5 px on 15x15, "
                                "sigma = 1 Gaussian noise"),
    "bulgedisk": dict(n=8192, desc="8192 Sersic bulge + exponential disk galaxies (shared centre), 128x128, "
                                   "Moffat PSF 25x25, Poisson + read noise"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_batch(workload: str, n: int, seed: int):
    """Draw, render with the HIP forward model at unit flux, add noise."""
    b = S.draw(workload, n, seed=seed)
    gm = G.Model.from_spec(S.MODEL_SPECS[b.model])
    db = G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, np.zeros(b.npix, np.float32),
                 np.ones(b.npix, np.float32), b.psf)
    units = G.gm_model_image(gm, db, S.unit_truth(b)).cpu().numpy()
    S.finish(b, units)
    db.data = torch.from_numpy(b.data).to(db.device)
    db.sigma = torch.from_numpy(b.sigma).to(db.device)
    return b, gm, db


def flops_per_eval(b: S.Batch, p: int, npl: int):
    """Algorithmic FLOPs of one model evaluation per galaxy: direct convolution
    of npl planes (2 H W K^2 npl, FP32) and the normal equations
    (2 H W (p(p+1)/2 + p + 1), FP64)."""
    hw = b.h.astype(np.float64) * b.w
    k2 = b.psf_k.astype(np.float64) ** 2
    return 2.0 * hw * k2 * npl, 2.0 * hw * (p * (p + 1) / 2 + p + 1)


def cpu_baseline(workload: str, n_sample: int, seed: int, gm: G.Model):
    """FP64 oracle on galaxies 0..n_sample-1 of the workload (images rendered by
    the oracle), all host cores, each side from its own moment-based start; the
    GPU fit of the same data gives the parity count."""
    import oracle as O
    from tests.gpu_helpers import oracle_batch, param_parity
    from tests.oracle_models import from_spec

    ncores = len(os.sched_getaffinity(0))
    b = oracle_batch(workload, n_sample, seed=seed)
    om = from_spec(b.model)
    db = G.Batch(b.h, b.w, b.img_off, b.psf_k, b.psf_off, b.data, b.sigma, b.psf)
    t0 = time.perf_counter()
    ostart, _ = O.default_guess_batch(om, b.h, b.w, b.img_off, b.data, b.sigma)
    rp, rc, rn, rs = O.fit_batch(om, b.h, b.w, b.img_off, b.data, b.sigma, b.psf_k, b.psf_off, b.psf, ostart,
                                 nthreads=ncores)
    dt = time.perf_counter() - t0
    start, _ = G.gm_default_guess(gm, db)
    gp, gc, gn, gs = [t.cpu().numpy() for t in G.gm_fit_batch(gm, db, start)]
    names = S.MODEL_SPECS[b.model]["names"]
    both = (gs == 0) & (rs == 0)
    npass = 0
    for g in np.where(both)[0]:
        ok, _ = param_parity(names, gp[g], rp[g], sky_sigma=float(np.median(b.image(b.sigma, g))))
        npass += int(ok.all())
    return dict(value=n_sample / dt, unit="galaxies/s", cores=ncores, kind="oracle",
                sample=f"galaxies 0..{n_sample - 1} of the workload (oracle-rendered), moment-based start and LM, "
                       f"{dt:.1f} s"), dict(sample=n_sample, both_converged=int(both.sum()), pass_1e4=npass,
                                                    oracle_converged=int((rs == 0).sum()),
                                                    gpu_converged=int((gs == 0).sum()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uneven", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=None, help="galaxies (default: the workload's size)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=48, help="oracle sample size (0 = skip)")
    ap.add_argument("--calib", action="store_true",
                    help="first run one 1 GiB device copy (reference for memory-traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the fitter shards by galaxy with no communication, "
              "and multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1073741824 bytes read, 1073741824 bytes written")
        del src, dst
    wl = WORKLOADS[args.workload]
    n = args.n or wl["n"]
    t0 = time.perf_counter()
    b, gm, db = make_batch(args.workload, n, args.seed)
    log(f"generated {n} galaxies ({b.npix / 1e6:.1f} Mpx) in {time.perf_counter() - t0:.1f} s")
    p = gm.p
    npl = p   # planes: model + every non-sky variable
    f_conv, f_red = flops_per_eval(b, p, npl)

    stream = torch.cuda.current_stream()
    params = torch.empty(n, p, dtype=torch.float64, device=db.device)
    chi2 = torch.empty(n, dtype=torch.float64, device=db.device)
    niter = torch.empty(n, dtype=torch.int32, device=db.device)
    status = torch.empty(n, dtype=torch.int32, device=db.device)
    err = torch.empty(n, p, dtype=torch.float64, device=db.device)
    ctx = G.context()

    def step(events=None):
        if events:
            events[0].record(stream)
        guess, _ = G.gm_default_guess(gm, db, ctx=ctx)
        if events:
            events[1].record(stream)
        G.gm_fit_batch(gm, db, guess, ctx=ctx, out=(params, chi2, niter, status))
        if events:
            events[2].record(stream)
        e = G.gm_param_errors(gm, db, params, ctx=ctx)
        if events:
            events[3].record(stream)
        return e

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {wall:.3f} s")
    fit_ms = [evs[i][1].elapsed_time(evs[i][2]) for i in range(args.steps)]
    guess_ms = [evs[i][0].elapsed_time(evs[i][1]) for i in range(args.steps)]
    err_ms = [evs[i][2].elapsed_time(evs[i][3]) for i in range(args.steps)]
    nit = niter.cpu().numpy()
    st = status.cpu().numpy()
    evals = (1 + nit.astype(np.float64)) * (st != G.ST_NONFINITE)
    flops_fit = float(np.sum((f_conv + f_red) * evals))
    fit_s = float(np.mean(fit_ms)) / 1e3
    achieved = flops_fit / fit_s / 1e12
    ms_step = wall / args.steps * 1e3
    value = n / (wall / args.steps)

    cpu, parity = None, None
    if args.cpu_sample > 0:
        log(f"cpu baseline: oracle on {args.cpu_sample} galaxies")
        cpu, parity = cpu_baseline(args.workload, args.cpu_sample, args.seed, gm)

    out = {
        "metric": "galaxies fitted/s at <=1e-4 rel param err vs oracle; learned-init vs plain LM",
        "value": value,
        "unit": "galaxies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "n_gal": n, "init": "default (moments)",
                   "max_iter": 100, "step_tol": 1e-4},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": (TRAFFIC.get(kernel_hash()) if (args.workload == "uneven" and n == 8192
                                                               and args.seed == 0) else None),
                     "traffic_unit": "bytes per launch",
                     "kernel": "lm_fit_kernel", "kernel_ms": fit_s * 1e3,
                     "flops_per_launch": flops_fit},
        "breakdown_ms": {"default_guess": float(np.mean(guess_ms)), "lm_fit": float(np.mean(fit_ms)),
                         "param_errors": float(np.mean(err_ms))},
        "lm": {"mean_iters": float(nit.mean()), "status_hist": np.bincount(st, minlength=4).tolist()},
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
