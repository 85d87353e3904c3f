#!/usr/bin/env python3
"""Throughput of the MLBA deblurring iteration on one MI355X.

A step is one full iteration of eq. (MLBA2) -- threshold + synthesis, blur and
residual, spectral preconditioner, adjoint blur, analysis + Bregman update --
on the 2048 x 2048 throughput workload (31 x 31 out-of-focus disk PSF,
rectangular blur model, 2078 x 2078 unknown, BCCB preconditioner with
alpha = 0.02, 3-level framelet, 25 bands).  Inputs are synthetic (seeded
scene, PSF and noise) and resident in HBM before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line: Mpixel-iter/s over the observed pixels, the
per-phase breakdown measured with HIP events on the library's stream during
the timed region, the roofline of the dominant kernel, and the FP64 oracle
timed on the host cores over a bounded sample of the same workload.  Two
sections follow: 64 uneven images batched under a hipGraph against 64
sequential solves, and the forward / backward time of 30 unrolled
iterations over 16 images of 256^2 with their gradients.
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
FP32_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, non-packed FP32

# HBM traffic of the dominant kernel per launch, from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) over `python bench.py
# --traffic-probe`, each scaled by what the counter reads for a plain 256 MiB
# copy on the same run (FETCH_SIZE 131,084 KiB -> x2.000, WRITE_SIZE
# 262,144 KiB -> x1.000).  The figure belongs to the kernel sources it was
# taken with: when their hash differs it is reported as null.
TRAFFIC = {
    ("blur_t", "implicit"): {"fetch_kib": 17573.7, "write_kib": 16878.0, "fetch_scale": 2.0, "write_scale": 1.0,
                             "sources_sha256": "fc757902bc5c941b6e9070e111ccee7e6f5d1340d05ffa7944585ad07c031ca3"},
}
TRAFFIC_SOURCES = ("paper_1504_07234_amd/csrc/conv.hip", "paper_1504_07234_amd/csrc/common.hpp",
                   "paper_1504_07234_amd/csrc/kernels.hpp")


def measured_traffic(phase: str, state: str):
    """Bytes per launch from the recorded counter passes, or None when none
    were taken for this kernel or its sources changed since."""
    import hashlib
    rec = TRAFFIC.get((phase, state))
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])


def phase_model(n, p, N, B, L, implicit):
    """Algorithmic bytes and flops of each phase of one iteration (float32).

    Explicit state z ([B][N][N]):
      synthesis : read z (B N^2), write u (N^2)
      blur_t    : read t (n^2), write w (N^2); 2 p^2 n^2 flops
      analysis  : read w (N^2), read and write z (2 B N^2)
    Implicit state omega (N x N, z = W omega):
      synthesis : L-1 low-pass levels (read + write N^2 each), then L levels
                  (read the level's low-pass, read the level above's output
                  except at the top, write N^2)
      blur_t    : read t (n^2), read and write omega (2 N^2); 2 p^2 n^2 flops
      analysis  : none
    Both:
      blur      : read u (N^2), read g (n^2), write r (n^2); 2 p^2 n^2 flops
      precond   : read r (n^2), write t (n^2)
    """
    f4 = 4.0
    if implicit:
        syn = f4 * N * N * (2 * (L - 1) + 2 + 3 * (L - 1))
        bt = f4 * (n * n + 2 * N * N)
        ana = 0.0
    else:
        syn = f4 * (B * N * N + N * N)
        bt = f4 * (n * n + N * N)
        ana = f4 * (N * N + 2 * B * N * N)
    return {
        "synthesis": {"bytes": syn, "flops": 0.0},
        "blur": {"bytes": f4 * (N * N + 2 * n * n), "flops": 2.0 * p * p * n * n},
        "precond": {"bytes": f4 * (2 * n * n), "flops": 0.0},
        "blur_t": {"bytes": bt, "flops": 2.0 * p * p * n * n},
        "analysis": {"bytes": ana, "flops": 0.0},
    }


def cpu_baseline(w, g64, delta, iters):
    """The FP64 oracle, as it stands, on `iters` iterations of the same
    workload (bounded sample)."""
    import numpy as np
    from oracle import mlba as omlba

    alphas = np.full(iters, w.alpha0)
    deltas = np.full(iters + 1, delta)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    omlba.mlba(g64, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, iters)
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    cores = max(1, int(round(cpu / wall)))
    return {
        "value": w.n * w.n * iters / wall / 1e6,
        "unit": "Mpixel-iter/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{iters} FP64 iterations of the {w.name} workload ({w.n}x{w.n} observed, "
                  f"{w.N}x{w.N} unknown, p={w.p}, {w.levels} levels) in {wall:.1f} s",
    }


def batched_section(count: int = 64, iters: int = 100):
    """64 uneven images (sides 128..1024, Gaussian PSFs 9..25, own alpha and
    noise), 2 levels, `iters` iterations: one batched hipGraph replay (tile
    shapes picked by the library's autotuner) against 64 sequential
    single-image restorations on the same stream."""
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
        deltas.append(0.9 / max(pl.opnorm(w.alpha0, 50), 0.9))
    outs = [torch.empty(pl.N, pl.N, device="cuda") for pl in plans]
    torch.cuda.synchronize()
    # 64 sequential plain solves (eager launches)
    for pl, g, a, d, o in zip(plans, gs, alphas, deltas, outs):  # warm-up
        pl.restore(g, alpha=a, mu=1e-3, delta=d, iters=2, out=o, track=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, g, a, d, o in zip(plans, gs, alphas, deltas, outs):
        pl.restore(g, alpha=a, mu=1e-3, delta=d, iters=iters, out=o, track=False)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    seq_ref = [o.clone() for o in outs]
    # batched: autotune the tile shapes, capture once, then time a replay
    batch = mlba.Batch(plans, max_iters=iters)
    tuned = batch.autotune(reps=5)
    batch.restore(gs, alpha=alphas, mu=1e-3, delta=deltas, iters=iters, outs=outs, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.restore(gs, alpha=alphas, mu=1e-3, delta=deltas, iters=iters, outs=outs, use_graph=True)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    identical = all(torch.equal(a, b) for a, b in zip(outs, seq_ref))
    px = sum(w.n * w.n for w in ws)
    batch.close()
    for pl in plans:
        pl.close()
    return {
        "images": count, "iters": iters, "observed_pixels": px,
        "sides": sorted({w.n for w in ws}),
        "batched_graph_s": round(t_bat, 5), "sequential_s": round(t_seq, 5),
        "speedup": round(t_seq / t_bat, 3),
        "batched_Mpx_it_s": round(px * iters / t_bat / 1e6, 1),
        "sequential_Mpx_it_s": round(px * iters / t_seq / 1e6, 1),
        "identical_to_sequential": identical,
        "autotuned": {"conv_rows": tuned["conv_rows"], "fft_rows_cap": tuned["fft_rows_cap"],
                      "fft_cols_cap": tuned["fft_cols_cap"]},
    }


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
    delta = 0.9 / max(U.plans[0].opnorm(w0.alpha0, 50), 0.9)
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
    discrepancy stop."""
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
    return out


def alg2_section(w, g, delta, steps: int = 10):
    """Algorithm 2 (section 4.2) on the 2048^2 rectangular workload: the
    preconditioner replaced by at most 5 PCG steps (tolerance 1e-3) on
    (A A^T + alpha I) t = r, preconditioned by the BCCB (C C^T + alpha I)^{-1};
    implicit state, `steps` timed iterations (one host read per PCG step)."""
    import torch

    from paper_1504_07234_amd import mlba

    psf = torch.as_tensor(w.psf, dtype=torch.float32).cuda()
    n = w.n
    with mlba.Plan(n, w.p, w.bc, w.precond, w.levels, psf) as plan:
        N = plan.N
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
    return {"model": "rect", "precond": "bccb", "alpha": w.alpha0, "pcg": [5, 1e-3], "steps": steps,
            "ms_per_step": round(el * 1e3 / steps, 5), "Mpx_it_s": round(n * n * steps / el / 1e6, 2),
            "pcg_steps": info.pcg_steps}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="rect-bccb-2048")
    ap.add_argument("--cpu-iters", type=int, default=3, help="oracle iterations for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-sequential section")
    ap.add_argument("--no-unrolled", action="store_true", help="skip the unrolled forward/backward section")
    ap.add_argument("--no-alg4", action="store_true", help="skip the Algorithm 4 / 4-NS and Algorithm 2 sections")
    ap.add_argument("--state", choices=("implicit", "explicit"), default="implicit",
                    help="iteration state: omega (z = W omega recomputed) or the frame coefficients z")
    ap.add_argument("--compare-steps", type=int, default=20,
                    help="iterations timed with the other state, for comparison (0: skip)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only two 256 MiB device copies x3 (counter calibration: the runtime copy and "
                         "a one-float-per-lane copy) and 3 iterations of the workload, for rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE passes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is described in DESIGN.md, not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_1504_07234_amd import mlba

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
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
    opn = plan.opnorm(w.alpha0, 50)
    delta = 0.9 / max(opn, 0.9)
    f = torch.empty((N, N), dtype=torch.float32, device="cuda")

    def run(implicit, steps, warmup, profile):
        st = torch.zeros((N, N) if implicit else (B, N, N), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=warmup, z=st, out=f, track=False,
                     implicit=implicit)
        torch.cuda.synchronize()
        if profile:
            plan.profile_begin(steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=steps, k0=warmup, z=st, out=f, track=False,
                     implicit=implicit)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ph = plan.profile_end() if profile else None
        _, info = plan.restore(g, alpha=w.alpha0, mu=w.mu, delta=delta, iters=1, k0=warmup + steps, z=st, out=f,
                               track=True, implicit=implicit)
        assert np.isfinite(info.rnorm[0]), "non-finite residual"
        return el, ph

    implicit = args.state == "implicit"
    blur_choice = None
    if not args.traffic_probe:
        # what the plan autotuner measures for the blur (direct taps vs FFT grid); the
        # timed run keeps the direct blur, whose VALU roofline is reported below
        blur_choice = plan.autotune(reps=5)
        plan.set_blur(mlba.BLUR_DIRECT)
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
    # ---- warmup, then the timed region: K iterations, phase events on the library stream --
    elapsed, (phases, rec) = run(implicit, args.steps, args.warmup, True)
    compare = None
    alt_blur = None
    if args.compare_steps > 0:
        el2, _ = run(not implicit, args.compare_steps, 3, False)
        compare = {"state": "explicit z" if implicit else "implicit omega", "steps": args.compare_steps,
                   "ms_per_step": round(el2 * 1e3 / args.compare_steps, 5),
                   "Mpx_it_s": round(n * n * args.compare_steps / el2 / 1e6, 2)}
        if blur_choice is not None and blur_choice["fft_ms"] is not None:
            # the same iteration with A and A^T evaluated on the FFT grid
            plan.set_blur(mlba.BLUR_FFT)
            el3, _ = run(implicit, args.compare_steps, 3, False)
            plan.set_blur(mlba.BLUR_DIRECT)
            alt_blur = {"blur": "fft", "steps": args.compare_steps,
                        "ms_per_step": round(el3 * 1e3 / args.compare_steps, 5),
                        "Mpx_it_s": round(n * n * args.compare_steps / el3 / 1e6, 2)}

    ms_per_step = elapsed * 1e3 / args.steps
    value = n * n * args.steps / elapsed / 1e6
    model = phase_model(n, p, N, B, w.levels, implicit)
    phase_out = {}
    for ph, (ms, launches) in phases.items():
        per_iter_ms = ms / max(rec, 1)
        b, fl = model[ph]["bytes"], model[ph]["flops"]
        phase_out[ph] = {
            "ms_per_iter": round(per_iter_ms, 4),
            "launches_per_iter": launches // max(rec, 1),
            "GBs": round(b / (per_iter_ms * 1e-3) / 1e9, 1) if per_iter_ms > 0 and b > 0 else None,
            "TFLOPs": round(fl / (per_iter_ms * 1e-3) / 1e12, 2) if fl and per_iter_ms > 0 else None,
        }
    def roofline_of(ph):
        """Roofline of the phase's main kernel from the live event times."""
        ms_iter = phases[ph][0] / max(rec, 1)
        nl = max(1, phases[ph][1] // max(rec, 1))
        if ph == "blur":  # conv + one tiny reduction launch: the conv is the kernel
            nl = 1
        launch_ms = ms_iter / nl
        if model[ph]["flops"] > 0:
            ach = model[ph]["flops"] / nl / (launch_ms * 1e-3) / 1e12
            r = {"bound": "alu", "achieved": round(ach, 2), "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": round(ach / FP32_VALU_PEAK_TFLOPS, 4), "traffic": measured_traffic(ph, args.state)}
        else:
            ach = model[ph]["bytes"] / nl / (launch_ms * 1e-3) / 1e9
            r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(ph, args.state)}
        r["kernel_phase"] = ph
        r["launch_ms"] = round(launch_ms, 4)
        r["algorithmic_bytes"] = round(model[ph]["bytes"] / nl)
        return r

    # dominant kernel: the longest single launch of an iteration
    def launch_ms(ph):
        per_iter = max(1, phases[ph][1] // max(rec, 1))
        if phases[ph][1] == 0:
            return 0.0
        return phases[ph][0] / max(rec, 1) / (1 if ph == "blur" else per_iter)

    dom = max(phases, key=launch_ms)
    roof = roofline_of(dom)
    roof_hbm = roofline_of("synthesis" if implicit else "analysis")
    total_bytes = sum(m["bytes"] for m in model.values())
    hbm_frac = (total_bytes / (HBM_PEAK_GBS * 1e9)) / (ms_per_step * 1e-3)

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
                   "delta": round(delta, 6), "state": "implicit omega (z = W omega)" if implicit else "explicit z"},
        "hbm_roofline_frac_whole_step": round(hbm_frac, 4),
        "phases": phase_out,
        "roofline": roof,
        "roofline_hbm": roof_hbm,
        "other_state": compare,
        "blur_autotune": blur_choice,
        "fft_blur_iteration": alt_blur,
    }
    plan.close()
    if not args.no_batched:
        out["batched"] = batched_section()
    if not args.no_unrolled:
        out["unrolled"] = unrolled_section()
    if not args.no_alg4:
        out["alg4"] = alg4_section(w, g, float(w.noise_level * blurred.double().norm()))
        out["alg2"] = alg2_section(w, g, delta)
    if not args.no_cpu:
        from oracle import blur as oblur
        g64 = synth.add_noise(oblur.blur(w.truth, w.psf, oblur.RECT), w.xi, w.noise_level)
        out["cpu_baseline"] = cpu_baseline(w, g64, delta, args.cpu_iters)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
