#!/usr/bin/env python3
"""Throughput of the MLBA deblurring iteration on one MI355X.

A step is one full iteration of eq. (MLBA2) -- threshold + synthesis, blur and
residual, spectral preconditioner, adjoint blur, analysis + Bregman update --
on the 2048 x 2048 throughput workload (31 x 31 out-of-focus disk PSF,
rectangular blur model, 2078 x 2078 unknown, BCCB preconditioner with
alpha = 0.02, 3-level framelet, 25 bands).  Inputs are synthetic (seeded
scene, PSF and noise) and resident in HBM before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

The blur is the one the plan autotuner picks (direct taps or the FFT grid).
Prints one JSON line: Mpixel-iter/s over the observed pixels, the per-kernel
and per-phase breakdown measured with HIP events on the library's stream on
every 4th iteration of the timed region, the roofline of the dominant kernel
(the one with the largest share of the iteration), and the FP64 oracle timed
on the host cores over a bounded sample of the same workload, and the FP32
transforms' error against FP64.  Sections follow: 64 uneven images batched
under a hipGraph against 64 sequential solves (implicit state and frame
coefficients); the forward / backward time of 30 unrolled iterations over 16
images of 256^2 with their gradients; Algorithm 4 and 4-NS (section 5) and
Algorithm 2 (section 4.2) on the 2048^2 observation; eq. (MLBA2) on the square
boundary models of Table 1; and the antireflective model (section 2.2).
"""
from __future__ import annotations

import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLBA Mpixel-iter/s at 2048² FP32 (% HBM roofline); batched vs plain; bwd/fwd ratio"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # published FP32 vector peak (packed FMA: 256 CU x 4 SIMD x 16 lanes x 4 x 2.4 GHz)
FP32_VALU_PEAK_TFLOPS = 78.6   # non-packed FP32 (2 flop per lane per FMA), the peak of code built without packed FP32
PROFILE_EVERY = 4              # kernel events on every 4th timed iteration (their overhead stays below 1 %)

# HBM traffic of the dominant kernel per iteration, from two rocprofv3 --pmc
# passes (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, summed over the
# kernel's launches in one iteration) over `python bench.py --traffic-probe`,
# each scaled by what the counter reads for a plain 256 MiB copy on the same run
# (FETCH_SIZE x2.000, WRITE_SIZE x1.000).  A figure belongs to the kernel sources
# it was taken with: when their hash differs it is reported as null.
TRAFFIC = {
    # 2078^2, 3 levels: the three shrink-synthesis launches of one iteration (d = 4, 2, 1)
    ("shrink_synthesis", "fft-implicit"): {
        "fetch_kib": 43445.9, "write_kib": 50610.5, "fetch_scale": 2.0, "write_scale": 1.0, "launches": 3,
        "sources_sha256": "665fbf6605b9a5faa8a04d7e0780ec5e11622f280cde6b5f55668b05c3c17a88"},
    # the direct A^T accumulating into omega (p = 31), one launch per iteration
    ("conv_blur_t", "direct-implicit"): {
        "fetch_kib": 17582.1, "write_kib": 16878.0, "fetch_scale": 2.0, "write_scale": 1.0, "launches": 1,
        "sources_sha256": "0cadeb24c27af3e487dec833b4026d5eb191001033c0a4f11b519d67bc769782"},
}
# the sources that define each kernel's device code
TRAFFIC_SOURCES = {
    "shrink_synthesis": ("shrink.hip", "framelet.hpp", "common.hpp"),
    "lowpass_level": ("shrink.hip", "framelet.hpp", "common.hpp"),
    "conv_blur_t": ("conv.hip", "common.hpp", "kernels.hpp"),
    "conv_blur": ("conv.hip", "common.hpp", "kernels.hpp"),
    "fc_cols": ("fftconv.hip", "fft_core.hpp", "common.hpp"),
    "fc_rows_fwd": ("fftconv.hip", "fft_core.hpp", "common.hpp"),
    "fc_rows_inv": ("fftconv.hip", "fft_core.hpp", "common.hpp"),
    "fc_residual_precond_rows": ("fftconv.hip", "fft_core.hpp", "common.hpp"),
    "precond_rows_fc_fwd": ("fftconv.hip", "fft_core.hpp", "common.hpp"),
    "fft_cols": ("fft.hip", "fft_core.hpp", "common.hpp"),
}


def direct_cols(p: int) -> bool:
    """PSF sizes whose FFT-grid column pass is the compiled p-tap convolution
    along y (the library's fftconv_direct_taps)."""
    return p in (5, 9, 17, 31)


def sources_hash(kernel: str):
    import hashlib
    files = TRAFFIC_SOURCES.get(kernel)
    if files is None:
        return None
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1504_07234_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, key: str):
    """HBM bytes per launch from the recorded counter passes, or None when none
    were taken for this kernel and configuration or its sources changed since."""
    rec = TRAFFIC.get((kernel, key))
    if rec is None or sources_hash(kernel) != rec["sources_sha256"]:
        return None
    per_iter = 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])
    return per_iter / rec["launches"]


def fft_grid(N: int) -> int:
    """Side of the FFT-blur grid: the smallest even 2^a 3^b >= N (at most 3072)."""
    best = 0
    a = 1
    while (1 << a) <= 3072:
        m = 1 << a
        while m <= 3072:
            if m >= N and (best == 0 or m < best):
                best = m
            m *= 3
        a += 1
    return best


def kernel_model(n, p, N, L, implicit, fft_blur):
    """Algorithmic bytes and flops of each kernel per iteration (float32
    values, complex = 8 bytes), and the roof that bounds it.

      synthesis_level   (z)     level: read 8 bands + low-pass, write N^2; 79 flops
                                per pixel: 9 thresholds 27, y-synthesis 39,
                                x-synthesis 13
      lowpass_level     (omega) level: read + write N^2; levels 1 and 2 in one
                                launch (read omega, write both planes)
      shrink_synthesis  (omega) level: read the level's low-pass and the level
                                above's output (not at the top), write N^2;
                                119 flops per pixel (FMA = 2): x-analysis 10,
                                y-analysis 30, 9 thresholds 27, y-synthesis 39,
                                x-synthesis 13
      conv_blur                 read u (N^2) and g, write r; 2 p^2 n^2 flops
      conv_blur_t               read t, write w (omega: read + write); 2 p^2 n^2
      fft_rows_fwd / _inv       n^2 reals <-> (n/2+1) n complex (transposed)
      fft_cols                  read + write (n/2+1) n complex, read the filter
      fc_rows_fwd (A)           read u (N^2), write (M/2+1) N complex
      fc_cols (A, A^T)          read the nonzero rows ((M/2+1) N, (M/2+1) n)
                                and write the kept ones ((M/2+1) n, (M/2+1) N);
                                with compiled taps (p = 5, 9, 17, 31) a p-tap
                                convolution along y reading the (M/2+1) p
                                taps, else the transform pair reading the PSF
                                spectrum and writing (M/2+1) M
      fc_rows_inv (A^T)         read (M/2+1) N complex, write w (omega: +read)
      fc_residual_precond_rows  read (M/2+1) n complex and g, write (n/2+1) n
      precond_rows_fc_fwd       read (n/2+1) n complex, write (M/2+1) n
      analysis_level    (z)     read v, read + write 8 bands, write low-pass; 48
                                flops per pixel: x-filters 10, y-filters 30,
                                8 accumulations
    """
    f4, c8 = 4.0, 8.0
    nn, NN = n * n, N * N
    hp = (n // 2 + 1) * n
    conv_fl = 2.0 * p * p * n * n
    m = {}
    if implicit:
        if L >= 3:  # levels 1 and 2 in one pass (read omega, write two planes), then one launch per level
            m["lowpass_level"] = {"bytes": f4 * NN * (3 + 2 * (L - 3)), "flops": 8.0 * NN * (L - 1), "launches": L - 2}
        else:
            m["lowpass_level"] = {"bytes": f4 * 2 * NN, "flops": 8.0 * NN, "launches": 1}
        m["shrink_synthesis"] = {"bytes": f4 * NN * (3 * L - 1), "flops": 119.0 * NN * L, "launches": L}
    else:
        m["synthesis_level"] = {"bytes": f4 * 10 * NN * L, "flops": 79.0 * NN * L, "launches": L}
        m["analysis_level"] = {"bytes": f4 * NN * (18 * L + 1), "flops": 48.0 * NN * L, "launches": L}
    if fft_blur:
        M = fft_grid(N)
        hm = M // 2 + 1
        m["fc_rows_fwd"] = {"bytes": f4 * NN + c8 * hm * N, "flops": 0.0, "launches": 1}
        if direct_cols(p):
            m["fc_cols"] = {"bytes": 2 * c8 * hm * (N + n) + 2 * c8 * hm * p, "flops": 8.0 * p * hm * (N + n),
                            "launches": 2}
        else:
            m["fc_cols"] = {"bytes": c8 * hm * (N + n) + 2 * 2 * c8 * hm * M, "flops": 0.0, "launches": 2}
        m["fc_residual_precond_rows"] = {"bytes": c8 * hm * n + f4 * nn + c8 * hp, "flops": 0.0, "launches": 1}
        m["fft_cols"] = {"bytes": 2 * c8 * hp + f4 * hp, "flops": 0.0, "launches": 1}
        m["precond_rows_fc_fwd"] = {"bytes": c8 * hp + c8 * hm * n, "flops": 0.0, "launches": 1}
        m["fc_rows_inv"] = {"bytes": c8 * hm * N + f4 * NN * (2 if implicit else 1), "flops": 0.0, "launches": 1}
    else:
        m["conv_blur"] = {"bytes": f4 * (NN + 2 * nn), "flops": conv_fl, "launches": 1}
        m["fft_rows_fwd"] = {"bytes": f4 * nn + c8 * hp, "flops": 0.0, "launches": 1}
        m["fft_cols"] = {"bytes": 2 * c8 * hp + f4 * hp, "flops": 0.0, "launches": 1}
        m["fft_rows_inv"] = {"bytes": c8 * hp + f4 * nn, "flops": 0.0, "launches": 1}
        m["conv_blur_t"] = {"bytes": f4 * (nn + (2 if implicit else 1) * NN), "flops": conv_fl, "launches": 1}
    m["reduce"] = {"bytes": 0.0, "flops": 0.0, "launches": 1}
    for k, v in m.items():  # the roof that binds at the published peaks
        t_hbm = v["bytes"] / (HBM_PEAK_GBS * 1e9)
        t_alu = v["flops"] / (FP32_PEAK_TFLOPS * 1e12)
        v["bound"] = "alu" if t_alu > t_hbm else "hbm"
    return m


def host_cpu():
    """Logical CPUs of this host and the processor model (lscpu)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return os.cpu_count(), model


def cpu_baseline(w, g64, delta, iters):
    """The FP64 oracle, as it stands, on `iters` iterations of the same
    workload (bounded sample), once limited to one thread and once with every
    thread its libraries take (cores = CPU time / wall time)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import mlba as omlba

    alphas = np.full(iters, w.alpha0)
    deltas = np.full(iters + 1, delta)

    def timed():
        r0 = resource.getrusage(resource.RUSAGE_SELF)
        t0 = time.perf_counter()
        omlba.mlba(g64, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, iters)
        wall = time.perf_counter() - t0
        r1 = resource.getrusage(resource.RUSAGE_SELF)
        cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
        return {"value": round(w.n * w.n * iters / wall / 1e6, 4), "wall_s": round(wall, 2),
                "cores": max(1, int(round(cpu / wall)))}

    with threadpool_limits(limits=1):
        one = timed()
    allc = timed()
    host_cores, model = host_cpu()
    return {
        "value": allc["value"],
        "unit": "Mpixel-iter/s",
        "cores": allc["cores"],
        "kind": "oracle",
        "sample": f"{iters} FP64 iterations of the {w.name} workload ({w.n}x{w.n} observed, "
                  f"{w.N}x{w.N} unknown, p={w.p}, {w.levels} levels) in {allc['wall_s']:.1f} s "
                  f"(one thread: {one['wall_s']:.1f} s)",
        "single_thread": one,
        "all_core": allc,
        "host_cores": host_cores,
        "host_cpu": model,
    }


def fft_fp32_error(w, g64):
    """FP32 transforms against FP64: the 2048-point BCCB preconditioner and the
    blur on the 2304-point grid of the workload, each applied by the library
    to the observation (and to the scene) and by the oracle in FP64 (relative
    2-norm and maximum errors)."""
    import numpy as np
    import torch

    from oracle import blur as oblur
    from oracle import precond as opc
    from paper_1504_07234_amd import mlba

    def errs(a, b):
        a = np.asarray(a, dtype=np.float64)
        return {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                "max_rel": float(np.abs(a - b).max() / np.abs(b).max())}

    psf = torch.as_tensor(w.psf, dtype=torch.float32).cuda()
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, psf) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        gp = plan.apply_P(torch.as_tensor(g64, dtype=torch.float32).cuda(), w.alpha0).double().cpu().numpy()
        au = plan.apply_A(torch.as_tensor(w.truth, dtype=torch.float32).cuda()).double().cpu().numpy()
    g32 = np.asarray(np.float32(g64), dtype=np.float64)
    t32 = np.asarray(np.float32(w.truth), dtype=np.float64)
    return {"P_bccb_2048": errs(gp, opc.apply_bccb(g32, w.psf, w.alpha0)),
            f"A_fft_grid_{fft_grid(w.N)}": errs(au, oblur.blur(t32, w.psf, oblur.RECT))}


def batched_section(count: int = 64, iters: int = 100):
    """64 uneven images (sides 128..1024, Gaussian PSFs 9..25, own alpha and
    noise), 2 levels, `iters` iterations: one batched hipGraph replay (tile
    shapes picked by the library's autotuner) against 64 sequential
    single-image restorations on the same stream, for the implicit state
    (omega) and for the explicit one (z)."""
    import torch

    import synth
    from paper_1504_07234_amd import mlba

    ws = synth.batched_workloads(count=count, iters=iters)
    plans, gs, alphas, deltas = [], [], [], []
    for w in ws:
        pl = mlba.Plan(w.n, w.p, mlba.RECT, mlba.BCCB, w.levels, torch.as_tensor(w.psf, dtype=torch.float32).cuda())
        b = pl.apply_A(torch.as_tensor(w.truth, dtype=torch.float32).cuda())
        xi = torch.as_tensor(w.xi, dtype=torch.float32).cuda()
        g = (b + (w.noise_level * b.double().norm() / xi.double().norm()).float() * xi).contiguous()
        plans.append(pl)
        gs.append(g)
        alphas.append(w.alpha0)
        deltas.append(pl.auto_step(w.alpha0))
    outs = [torch.empty(pl.N, pl.N, device="cuda") for pl in plans]
    px = sum(w.n * w.n for w in ws)
    batch = mlba.Batch(plans, max_iters=iters)
    tuned = batch.autotune(reps=5)
    res = {"images": count, "iters": iters, "observed_pixels": px, "sides": sorted({w.n for w in ws}),
           "autotuned": {"conv_rows": tuned["conv_rows"], "fft_rows_cap": tuned["fft_rows_cap"],
                         "fft_cols_cap": tuned["fft_cols_cap"]}}
    for implicit in (True, False):
        # 64 sequential single-image solves (eager launches), the same state
        torch.cuda.synchronize()
        for pl, g, a, d, o in zip(plans, gs, alphas, deltas, outs):  # warm-up
            pl.restore(g, alpha=a, mu=1e-3, delta=d, iters=2, out=o, track=False, implicit=implicit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pl, g, a, d, o in zip(plans, gs, alphas, deltas, outs):
            pl.restore(g, alpha=a, mu=1e-3, delta=d, iters=iters, out=o, track=False, implicit=implicit)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        seq_ref = [o.clone() for o in outs]
        # batched: capture once, then time a replay (host submission: one graph launch)
        batch.restore(gs, alpha=alphas, mu=1e-3, delta=deltas, iters=iters, outs=outs, use_graph=True,
                      implicit=implicit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.restore(gs, alpha=alphas, mu=1e-3, delta=deltas, iters=iters, outs=outs, use_graph=True,
                      implicit=implicit)
        t_submit = time.perf_counter() - t0
        torch.cuda.synchronize()
        t_bat = time.perf_counter() - t0
        identical = all(torch.equal(a, b) for a, b in zip(outs, seq_ref))
        key = "implicit" if implicit else "explicit"
        res[key] = {
            "batched_graph_s": round(t_bat, 5), "sequential_s": round(t_seq, 5),
            "speedup": round(t_seq / t_bat, 3),
            "batched_Mpx_it_s": round(px * iters / t_bat / 1e6, 1),
            "sequential_Mpx_it_s": round(px * iters / t_seq / 1e6, 1),
            "host_submit_ms": round(t_submit * 1e3, 3),
            "identical_to_sequential": identical,
        }
    batch.close()
    for pl in plans:
        pl.close()
    return res


def unrolled_section(reps: int = 5):
    """Differentiable unrolled MLBA: 16 images of 256^2, 15 x 15 Gaussian PSF
    (sigma 2.5), 2 levels (17 thresholds), K = 30 iterations, checkpoints every
    5; loss ||f - f_true||^2.  Forward (with checkpoints) and backward (segment
    recompute + reverse sweep, gradients for mu, alpha, PSF and g) timed with
    HIP events on the library's stream, averaged over `reps` calls."""
    import torch

    import synth
    from paper_1504_07234_amd import mlba

    ws = synth.unrolled_workloads()
    w0 = ws[0]
    K, ce = w0.iters, w0.extra["ckpt_every"]
    psf = torch.as_tensor(w0.psf, dtype=torch.float32).cuda()
    U = mlba.Unrolled([w.n for w in ws], w0.p, w0.levels, psf, K, ce)
    gs, truths = [], []
    for w, pl in zip(ws, U.plans):
        truth = torch.as_tensor(w.truth, dtype=torch.float32).cuda()
        b = pl.apply_A(truth)
        xi = torch.as_tensor(w.xi, dtype=torch.float32).cuda()
        gs.append((b + (w.noise_level * b.double().norm() / xi.double().norm()).float() * xi).contiguous())
        truths.append(truth)
    delta = U.plans[0].auto_step(w0.alpha0)
    mu = [w0.mu] * U.bands
    fs, ck = U.forward(gs, alpha=w0.alpha0, mu=mu, delta=delta)
    dfs = [(2.0 * (f - t)).contiguous() for f, t in zip(fs, truths)]
    res = U.backward(gs, dfs, ck, alpha=w0.alpha0, mu=mu, delta=delta)  # warm-up
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_f = t_b = 0.0
    for _ in range(reps):
        ev[0].record()
        U.forward(gs, alpha=w0.alpha0, mu=mu, delta=delta, ckpts=ck, outs=fs)
        ev[1].record()
        res = U.backward(gs, dfs, ck, alpha=w0.alpha0, mu=mu, delta=delta)
        ev[2].record()
        torch.cuda.synchronize()
        t_f += ev[0].elapsed_time(ev[1])
        t_b += ev[1].elapsed_time(ev[2])
    t_f /= reps
    t_b /= reps
    finite = bool(torch.isfinite(res["mu"]).all() and torch.isfinite(res["psf"]).all()
                  and torch.isfinite(res["alpha"]))
    px = sum(w.n * w.n for w in ws)
    U.close()
    return {
        "images": len(ws), "n": w0.n, "p": w0.p, "levels": w0.levels, "bands": 8 * w0.levels + 1,
        "iters": K, "ckpt_every": ce, "alpha": w0.alpha0, "mu": w0.mu, "delta": round(delta, 6),
        "forward_ms": round(t_f, 4), "backward_ms": round(t_b, 4), "bwd_fwd_ratio": round(t_b / t_f, 3),
        "forward_Mpx_it_s": round(px * K / (t_f * 1e-3) / 1e6, 1),
        "grads": ["mu[17]", "alpha", "psf[15x15]", "g"], "grads_finite": finite,
    }


def alg4_section(w, g, noise, steps: int = 30):
    """Algorithm 4 (section 5) on the 2048^2 observation as a square model:
    periodic boundary conditions, C^T (C C^T + alpha I)^{-1} by FFT (no A^T
    product), implicit state, alpha = 0.02, unit step, `steps` timed
    iterations; and Algorithm 4-NS (q = 0.5, rho = 1e-4) run to its
    discrepancy stop, with that BCCB plan and with the DCT of the symmetrised
    PSF on the reflective model."""
    import torch

    from paper_1504_07234_amd import mlba

    psf = torch.as_tensor(w.psf, dtype=torch.float32).cuda()
    n = w.n
    out = {"model": "periodic", "precond": "bccb", "alpha": 0.02, "levels": w.levels, "state": "implicit omega"}
    with mlba.Plan(n, w.p, mlba.PERIODIC, mlba.BCCB, w.levels, psf) as plan:
        f = torch.empty((n, n), dtype=torch.float32, device="cuda")
        om = torch.zeros((n, n), dtype=torch.float32, device="cuda")
        plan.restore(g, alpha=0.02, mu=w.mu, delta=1.0, iters=3, z=om, out=f, track=False, implicit=True,
                     method=mlba.ALG4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.restore(g, alpha=0.02, mu=w.mu, delta=1.0, iters=steps, k0=3, z=om, out=f, track=False,
                     implicit=True, method=mlba.ALG4)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out.update({"steps": steps, "ms_per_step": round(el * 1e3 / steps, 5),
                    "Mpx_it_s": round(n * n * steps / el / 1e6, 2)})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = plan.restore(g, alpha=0.5, mu=w.mu, delta=1.0, iters=500, out=f, implicit=True,
                               method=mlba.ALG4, ns=(0.5, 1e-4), stop=(noise, 0.0, 1))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["ns"] = {"q": 0.5, "rho": 1e-4, "iters_to_stop": info.iters_done, "s_total": round(el, 5),
                     "ms_per_step": round(el * 1e3 / max(info.iters_done, 1), 5),
                     "last_alpha": info.alphas[-1] if info.alphas else None}
    # 4-NS with the DCT of the symmetrised PSF on the reflective model (the DCT
    # form of Example 4's Alg-BC4-NS)
    with mlba.Plan(n, w.p, mlba.REFLECT, mlba.DCT, w.levels, psf) as plan:
        blur = plan.autotune(reps=3)["blur"]  # the residual's A
        f = torch.empty((n, n), dtype=torch.float32, device="cuda")
        plan.restore(g, alpha=0.5, mu=w.mu, delta=1.0, iters=2, out=f, implicit=True, method=mlba.ALG4,
                     ns=(0.5, 1e-4), stop=(noise, 0.0, 1), track=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = plan.restore(g, alpha=0.5, mu=w.mu, delta=1.0, iters=500, out=f, implicit=True,
                               method=mlba.ALG4, ns=(0.5, 1e-4), stop=(noise, 0.0, 1))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["ns_dct"] = {"model": "reflective", "precond": "dct", "blur": blur, "q": 0.5, "rho": 1e-4,
                         "iters_to_stop": info.iters_done, "s_total": round(el, 5),
                         "ms_per_step": round(el * 1e3 / max(info.iters_done, 1), 5)}
    return out


def square_models_section(w, g, steps: int = 30):
    """Eq. (MLBA2) on the square models of Table 1 at 2048^2 (p = 31, L = 3,
    alpha = 0.02, implicit state, the library's automatic step, the blur the
    plan autotuner picks): zero and reflective pads with the BCCB
    preconditioner (Algorithm 1), the reflective pad with the DCT of the
    symmetrised PSF (Algorithm 3), and the periodic pad with the BCCB matrix
    (there A = C and the residual is formed in the spectrum)."""
    import torch

    from paper_1504_07234_amd import mlba

    psf = torch.as_tensor(w.psf, dtype=torch.float32).cuda()
    n = w.n
    out = []
    for bc, pc in (("zero", "bccb"), ("reflect", "bccb"), ("reflect", "dct"), ("periodic", "bccb")):
        BC = {"zero": mlba.ZERO, "reflect": mlba.REFLECT, "periodic": mlba.PERIODIC}[bc]
        PC = {"bccb": mlba.BCCB, "dct": mlba.DCT}[pc]
        with mlba.Plan(n, w.p, BC, PC, w.levels, psf) as plan:
            tune = plan.autotune(reps=3)
            delta = plan.auto_step(w.alpha0)
            f = torch.empty((n, n), dtype=torch.float32, device="cuda")
            om = torch.zeros((n, n), dtype=torch.float32, device="cuda")
            plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=3, z=om, out=f, track=False,
                         implicit=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=steps, k0=3, z=om, out=f, track=False,
                         implicit=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        out.append({"model": bc, "precond": pc, "blur": tune["blur"], "delta": round(delta, 6), "steps": steps,
                    "ms_per_step": round(el * 1e3 / steps, 5), "Mpx_it_s": round(n * n * steps / el / 1e6, 2)})
    return out


def alg2_section(w, g, delta, steps: int = 10):
    """Algorithm 2 (section 4.2) on the 2048^2 rectangular workload: the
    preconditioner replaced by at most 5 PCG steps (tolerance 1e-3) on
    (A A^T + alpha I) t = r, preconditioned by the BCCB (C C^T + alpha I)^{-1};
    implicit state, the autotuned blur, `steps` timed iterations (one host read
    per PCG step)."""
    import torch

    from paper_1504_07234_amd import mlba

    psf = torch.as_tensor(w.psf, dtype=torch.float32).cuda()
    n = w.n
    with mlba.Plan(n, w.p, w.bc, w.precond, w.levels, psf) as plan:
        N = plan.N
        blur = plan.autotune(reps=3)["blur"]  # each PCG step is one A A^T product
        f = torch.empty((N, N), dtype=torch.float32, device="cuda")
        om = torch.zeros((N, N), dtype=torch.float32, device="cuda")
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=2, z=om, out=f, track=False, implicit=True,
                     method=mlba.ALG2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=steps, k0=2, z=om, out=f,
                               implicit=True, method=mlba.ALG2)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    return {"model": "rect", "precond": "bccb", "blur": blur, "alpha": w.alpha0, "pcg": [5, 1e-3], "steps": steps,
            "ms_per_step": round(el * 1e3 / steps, 5), "Mpx_it_s": round(n * n * steps / el / 1e6, 2),
            "pcg_steps": info.pcg_steps}


def antireflective_section(steps: int = 30, warmup: int = 3):
    """Alg-BC3 of Example 4 at n = 1025: the antireflective model (its pad in
    A, the reblur A' in place of A^T; the autotuner picks the direct taps or
    the FFT grid, m = 1055 on a 1152 grid), the antireflective-transform
    preconditioner (three passes of complex FFTs of length 2(n - 1) = 2048),
    31 x 31 Gaussian, 3 levels, implicit state, automatic step; `steps` timed
    iterations with the per-kernel profile.  Algorithmic bytes of the
    transform passes: rows T^-1 read n^2 and write n^2 floats, columns read
    n^2 and the n^2 filter and write n^2, rows T read n^2 and write n^2; of the
    grid passes (A and A'): rows read n^2 and write the (M/2+1) x m half
    spectrum, columns read it and the PSF spectrum and write the (M/2+1) x n
    rows kept, inverse rows read those and read + write n^2 (on the grid the
    residual's inverse rows and the transform's forward rows are one launch:
    read the kept rows and g, write the n^2 transform rows).
    Alg-BC4 (Algorithm 4 with the same transform, no A' product) is timed on
    the same plan."""
    import torch

    import synth
    from paper_1504_07234_amd import mlba

    w = synth.make_workload("antireflect-ar-1025")
    n, p = w.n, w.p
    psf = torch.as_tensor(w.psf, dtype=torch.float32).cuda()
    with mlba.Plan(n, p, mlba.RECT, mlba.NONE, 1, psf) as rect:
        blurred = rect.apply_A(torch.as_tensor(w.truth, dtype=torch.float32).cuda())
    xi = torch.as_tensor(w.xi, dtype=torch.float32).cuda()
    g = (blurred + (w.noise_level * blurred.double().norm() / xi.double().norm()).float() * xi).contiguous()
    names = {"fft_rows_fwd": "ar_rows_fwd", "fft_cols": "ar_cols_filter", "fft_rows_inv": "ar_rows_inv",
             "fc_residual_precond_rows": "fc_residual_ar_rows"}
    with mlba.Plan(n, p, w.bc, w.precond, w.levels, psf) as plan:
        N = plan.N
        tune = plan.autotune(reps=5)
        delta = plan.auto_step(w.alpha0)
        f = torch.empty((N, N), dtype=torch.float32, device="cuda")
        om = torch.zeros((N, N), dtype=torch.float32, device="cuda")
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=warmup, z=om, out=f, track=False,
                     implicit=True)
        plan.profile_begin(steps, every=PROFILE_EVERY)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=steps, k0=warmup, z=om, out=f, track=False,
                     implicit=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        _, rec = plan.profile_end()
        kernels = plan.profile_kernels()
        # Alg-BC4 on the same plan: Q' (Q Q' + alpha I)^-1 r by the transform, no A' product
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=1.0, iters=warmup, z=om, out=f, track=False,
                     implicit=True, method=mlba.ALG4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=1.0, iters=steps, k0=warmup, z=om, out=f, track=False,
                     implicit=True, method=mlba.ALG4)
        torch.cuda.synchronize()
        el4 = time.perf_counter() - t0
    rec = max(rec, 1)
    fft_blur = tune["blur"] == "fft"
    model = kernel_model(n, p, N, w.levels, True, False)
    nn = 4.0 * n * n
    model["fft_rows_fwd"] = {"bytes": 2 * nn, "flops": 0.0, "launches": 1, "bound": "hbm"}
    model["fft_cols"] = {"bytes": 3 * nn, "flops": 0.0, "launches": 1, "bound": "hbm"}
    model["fft_rows_inv"] = {"bytes": 2 * nn, "flops": 0.0, "launches": 1, "bound": "hbm"}
    if fft_blur:
        m_ = n + p - 1
        M = fft_grid(m_)
        hm = M // 2 + 1
        for k in ("conv_blur", "conv_blur_t"):
            model.pop(k)
        model["fc_rows_fwd"] = {"bytes": 2 * (nn + 8.0 * hm * m_), "flops": 0.0, "launches": 2, "bound": "hbm"}
        if direct_cols(p):
            model["fc_cols"] = {"bytes": 2 * 8.0 * hm * (m_ + n) + 2 * 8.0 * hm * p,
                                "flops": 8.0 * p * hm * (m_ + n), "launches": 2, "bound": "hbm"}
        else:
            model["fc_cols"] = {"bytes": 2 * 8.0 * hm * (m_ + M + n), "flops": 0.0, "launches": 2, "bound": "hbm"}
        # the residual's inverse rows fused with the transform's forward rows: read the
        # kept half-spectrum rows and g, write Tr; the reblur's inverse rows into omega
        model["fc_residual_precond_rows"] = {"bytes": 8.0 * hm * n + 2 * nn, "flops": 0.0, "launches": 1,
                                             "bound": "hbm"}
        model.pop("fft_rows_fwd")
        model["fc_rows_inv"] = {"bytes": 8.0 * hm * n + 2 * nn, "flops": 0.0, "launches": 1, "bound": "hbm"}
    kern = {}
    for k, (ms, nl) in kernels.items():
        us = ms * 1e3 / rec
        e = {"us_per_iter": round(us, 2), "launches_per_iter": round(nl / rec, 2)}
        mk = model.get(k)
        if mk is not None and us > 0:
            e["GBs"] = round(mk["bytes"] / (us * 1e-6) / 1e9, 1)
            e["bound"] = mk["bound"]
            e["frac"] = round(e["GBs"] / HBM_PEAK_GBS if mk["bound"] == "hbm" else
                              mk["flops"] / (us * 1e-6) / 1e12 / FP32_PEAK_TFLOPS, 4)
        kern[names.get(k, k)] = e
    return {"workload": w.name, "n": n, "p": p, "levels": w.levels, "boundary": "antireflective (A' = reblur)",
            "precond": "antireflective transform (FFT length 2048)", "alpha": w.alpha0, "mu": w.mu,
            "delta": round(delta, 6), "state": "implicit omega", "steps": steps,
            "blur": f"fft grid {fft_grid(n + p - 1)}" if fft_blur else "direct taps",
            "blur_autotune": tune,
            "ms_per_step": round(el * 1e3 / steps, 5), "Mpx_it_s": round(n * n * steps / el / 1e6, 2),
            "alg4": {"ms_per_step": round(el4 * 1e3 / steps, 5), "Mpx_it_s": round(n * n * steps / el4 / 1e6, 2)},
            "kernels": kern}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="rect-bccb-2048")
    ap.add_argument("--cpu-iters", type=int, default=5, help="oracle iterations for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-sequential section")
    ap.add_argument("--no-unrolled", action="store_true", help="skip the unrolled forward/backward section")
    ap.add_argument("--no-alg4", action="store_true", help="skip the Algorithm 4 / 4-NS and Algorithm 2 sections")
    ap.add_argument("--no-ar", action="store_true", help="skip the antireflective (Alg-BC3) section")
    ap.add_argument("--only-ar", action="store_true",
                    help="run only the antireflective section and print its JSON (for profiling it alone)")
    ap.add_argument("--state", choices=("implicit", "explicit"), default="implicit",
                    help="iteration state: omega (z = W omega recomputed) or the frame coefficients z")
    ap.add_argument("--compare-steps", type=int, default=20,
                    help="iterations timed with the other state, for comparison (0: skip)")
    ap.add_argument("--blur", choices=("auto", "fft", "direct"), default="auto",
                    help="A and A^T: the plan autotuner's choice (default), the FFT grid or the direct taps")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only two 256 MiB device copies x3 (counter calibration: the runtime copy and "
                         "a one-float-per-lane copy) and 3 iterations of the workload, for rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE passes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path: independent images shard without communication, "
              "a single image would need halo exchanges and a distributed transpose)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_1504_07234_amd import mlba

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.only_ar:
        print(json.dumps({"antireflective": antireflective_section()}), flush=True)
        return 0
    w = synth.make_workload(args.workload)
    n, p = w.n, w.p

    # ---- inputs in HBM: scene, PSF, observed image g = A f + eta --------
    psf = torch.as_tensor(w.psf, dtype=torch.float32).cuda()
    plan = mlba.Plan(n, p, w.bc, w.precond, w.levels, psf)
    N, B = plan.N, plan.bands
    # the scene extends beyond the field of view: observe it through the rectangular blur
    with mlba.Plan(n, p, mlba.RECT, mlba.NONE, 1, psf) as rect:
        blurred = rect.apply_A(torch.as_tensor(w.truth, dtype=torch.float32).cuda())
    xi = torch.as_tensor(w.xi, dtype=torch.float32).cuda()
    g = blurred + (w.noise_level * blurred.double().norm() / xi.double().norm()).float() * xi
    g = g.contiguous()
    delta = plan.auto_step(w.alpha0)  # the library's automatic step (delta <= 0)
    f = torch.empty((N, N), dtype=torch.float32, device="cuda")

    def run(implicit, steps, warmup, profile):
        st = torch.zeros((N, N) if implicit else (B, N, N), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=warmup, z=st, out=f, track=False,
                     implicit=implicit)
        torch.cuda.synchronize()
        if profile:
            plan.profile_begin(steps, every=PROFILE_EVERY)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=steps, k0=warmup, z=st, out=f, track=False,
                     implicit=implicit)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = None
        if profile:
            phases, rec = plan.profile_end()
            prof = (phases, plan.profile_kernels(), rec)
        _, info = plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=1, k0=warmup + steps, z=st, out=f,
                               track=True, implicit=implicit)
        assert np.isfinite(info.rnorm[0]), "non-finite residual"
        return el, prof

    implicit = args.state == "implicit"
    blur_choice = None
    if not args.traffic_probe:
        # the plan autotuner times the direct blur against the FFT grid and keeps the faster
        blur_choice = plan.autotune(reps=5)
    if args.blur != "auto":
        plan.set_blur(mlba.BLUR_FFT if args.blur == "fft" else mlba.BLUR_DIRECT)
    if args.blur == "auto":
        fft_blur = blur_choice is None or blur_choice["blur"] == "fft"
        if blur_choice is None:
            plan.set_blur(mlba.BLUR_FFT)
    else:
        fft_blur = args.blur == "fft"
    if args.traffic_probe:
        src = torch.rand(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)  # runtime copy (wide requests)
        for _ in range(3):
            mlba.soft_threshold(src, 0.0, 1.0, out=dst)  # one float per lane: x = S_0(z) = z
        torch.cuda.synchronize()
        st = torch.zeros((N, N) if implicit else (B, N, N), dtype=torch.float32, device="cuda")
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=3, z=st, out=f, track=False, implicit=implicit)
        torch.cuda.synchronize()
        print("traffic probe done", flush=True)
        return 0
    # ---- warmup, then the timed region: K iterations, kernel events on the library stream --
    elapsed, (phases, kernels, rec) = run(implicit, args.steps, args.warmup, True)
    compare = None
    alt_blur = None
    if args.compare_steps > 0:
        el2, _ = run(not implicit, args.compare_steps, 3, False)
        compare = {"state": "explicit z" if implicit else "implicit omega", "steps": args.compare_steps,
                   "ms_per_step": round(el2 * 1e3 / args.compare_steps, 5),
                   "Mpx_it_s": round(n * n * args.compare_steps / el2 / 1e6, 2)}
        if args.blur == "auto" and blur_choice is not None and blur_choice["fft_ms"] is not None:
            # the same iteration with the blur the autotuner did not pick
            plan.set_blur(mlba.BLUR_DIRECT if fft_blur else mlba.BLUR_FFT)
            el3, _ = run(implicit, args.compare_steps, 3, False)
            plan.set_blur(mlba.BLUR_FFT if fft_blur else mlba.BLUR_DIRECT)
            alt_blur = {"blur": "direct" if fft_blur else "fft", "steps": args.compare_steps,
                        "ms_per_step": round(el3 * 1e3 / args.compare_steps, 5),
                        "Mpx_it_s": round(n * n * args.compare_steps / el3 / 1e6, 2)}

    ms_per_step = elapsed * 1e3 / args.steps
    value = n * n * args.steps / elapsed / 1e6
    model = kernel_model(n, p, N, w.levels, implicit, fft_blur)
    key = f"{'fft' if fft_blur else 'direct'}-{'implicit' if implicit else 'explicit'}"
    rec = max(rec, 1)
    kern_out = {}
    for k, (ms, nl) in kernels.items():
        us_iter = ms * 1e3 / rec
        mk = model.get(k)
        e = {"us_per_iter": round(us_iter, 2), "launches_per_iter": round(nl / rec, 2),
             "us_per_launch": round(ms * 1e3 / nl, 2)}
        if mk is not None and us_iter > 0:
            e["GBs"] = round(mk["bytes"] / (us_iter * 1e-6) / 1e9, 1)
            e["TFLOPs"] = round(mk["flops"] / (us_iter * 1e-6) / 1e12, 2) if mk["flops"] else None
            e["bound"] = mk["bound"]
            e["frac"] = round(e["GBs"] / HBM_PEAK_GBS if mk["bound"] == "hbm" else
                              e["TFLOPs"] / FP32_PEAK_TFLOPS, 4)
        kern_out[k] = e
    phase_out = {ph: {"us_per_iter": round(ms * 1e3 / rec, 2), "launches_per_iter": round(nl / rec, 2)}
                 for ph, (ms, nl) in phases.items()}

    # dominant kernel: the one that takes the largest share of the iteration
    dom = max((k for k in kernels if k in model), key=lambda k: kernels[k][0])
    mk = model[dom]
    ms, nl = kernels[dom]
    launch_s = ms * 1e-3 / nl
    per_launch_bytes = mk["bytes"] / mk["launches"]
    per_launch_flops = mk["flops"] / mk["launches"]
    if mk["bound"] == "alu":
        ach = per_launch_flops / launch_s / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_PEAK_TFLOPS, 4)}
    else:
        ach = per_launch_bytes / launch_s / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4)}
    # the same launch against the arithmetic roofs: the published FP32 peak
    # (packed FMA) and the non-packed peak of the library's code (built without packed FP32)
    tfl = per_launch_flops / launch_s / 1e12
    roof["alu"] = {"achieved_tflops": round(tfl, 2), "frac_published": round(tfl / FP32_PEAK_TFLOPS, 4),
                   "frac_nonpacked": round(tfl / FP32_VALU_PEAK_TFLOPS, 4)}
    roof["traffic"] = measured_traffic(dom, key)
    roof.update({"kernel": dom, "launch_us": round(launch_s * 1e6, 2), "launches_per_iter": mk["launches"],
                 "algorithmic_bytes_per_launch": round(per_launch_bytes),
                 "algorithmic_flops_per_launch": round(per_launch_flops),
                 "iterations_sampled": rec, "sampled_every": PROFILE_EVERY})
    total_bytes = sum(v["bytes"] for v in model.values())
    hbm_frac = (total_bytes / (HBM_PEAK_GBS * 1e9)) / (ms_per_step * 1e-3)
    # every kernel at its own roof: sum_k max(bytes_k / HBM peak, flops_k / FP32 peak)
    t_roof = sum(max(v["bytes"] / (HBM_PEAK_GBS * 1e9), v["flops"] / (FP32_PEAK_TFLOPS * 1e12))
                 for v in model.values())
    t_roof_np = sum(max(v["bytes"] / (HBM_PEAK_GBS * 1e9), v["flops"] / (FP32_VALU_PEAK_TFLOPS * 1e12))
                    for v in model.values())

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpixel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "p": p, "N": N, "levels": w.levels, "bands": B,
                   "boundary": "rect", "precond": "bccb", "alpha": w.alpha0, "mu": w.mu,
                   "delta": round(delta, 6), "state": "implicit omega (z = W omega)" if implicit else "explicit z",
                   "blur": f"fft grid {fft_grid(N)}" if fft_blur else "direct taps"},
        "hbm_roofline_frac_whole_step": round(hbm_frac, 4),
        "roofline_frac_whole_step": {"t_roof_us": round(t_roof * 1e6, 2), "t_meas_us": round(ms_per_step * 1e3, 2),
                                     "frac": round(t_roof / (ms_per_step * 1e-3), 4),
                                     "t_roof_nonpacked_us": round(t_roof_np * 1e6, 2),
                                     "frac_nonpacked": round(t_roof_np / (ms_per_step * 1e-3), 4)},
        "roofline": roof,
        "kernels": kern_out,
        "phases": phase_out,
        "other_state": compare,
        "blur_autotune": blur_choice,
        "other_blur": alt_blur,
    }
    plan.close()
    if not args.no_batched:
        out["batched"] = batched_section()
    if not args.no_unrolled:
        out["unrolled"] = unrolled_section()
    if not args.no_alg4:
        out["alg4"] = alg4_section(w, g, float(w.noise_level * blurred.double().norm()))
        out["alg2"] = alg2_section(w, g, delta)
        out["square_models"] = square_models_section(w, g)
    if not args.no_ar:
        out["antireflective"] = antireflective_section()
    if not args.no_cpu:
        from oracle import blur as oblur
        g64 = synth.add_noise(oblur.blur(w.truth, w.psf, oblur.RECT), w.xi, w.noise_level)
        out["cpu_baseline"] = cpu_baseline(w, g64, delta, args.cpu_iters)
        out["fft_fp32_error"] = fft_fp32_error(w, g64)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
