"""Reverse-mode gradient of K unrolled MLBA iterations on the GPU, against
the FP64 oracle adjoint (itself pinned by central finite differences).

The soft threshold is differentiated almost everywhere (0 at the kink), on
both sides.  Gradients are compared norm-wise: FP32 round-off over K steps
gives ~1e-5 relative; a coefficient whose |z| lies within round-off of its
threshold would flip one mask entry, which the 1e-3 bound absorbs.
"""
import concurrent.futures as cf
import multiprocessing as mp

import numpy as np
import pytest

import synth
from oracle import adjoint as oadj
from oracle import blur as oblur
from oracle import mlba as omlba
from tests._util import announce, cuda, host, observed, rel_err

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


def _images(sizes, p, seed, sigma=1.5):
    gen = synth.rng(seed)
    H = synth.gaussian_psf(p, sigma)
    out = []
    for n in sizes:
        truth = synth.shapes_image(n + p - 1, gen, n_rect=5, n_disk=3, n_bumps=2)
        g = synth.add_noise(oblur.blur(truth, H, oblur.RECT), synth.white_noise((n, n), gen), 0.01)
        out.append((g, truth))
    return H, out


def _oracle_sum(H, imgs, dfs, alpha, mu, delta, K, L):
    tot = None
    for (g, _), df in zip(imgs, dfs):
        gr = oadj.unrolled_grad(g, H, alpha, mu, delta, K, L, df)
        if tot is None:
            tot = {"mu": gr["mu"].copy(), "alpha": gr["alpha"], "psf": gr["psf"].copy(), "g": [gr["g"]],
                   "f": [gr["f"]]}
        else:
            tot["mu"] += gr["mu"]
            tot["alpha"] += gr["alpha"]
            tot["psf"] += gr["psf"]
            tot["g"].append(gr["g"])
            tot["f"].append(gr["f"])
    return tot


def _run(mlba, sizes, p, L, K, ce, H, imgs, dfs, alpha, mu, delta):
    with mlba.Unrolled(sizes, p, L, cuda(H), K, ce) as U:
        gs = [cuda(g) for g, _ in imgs]
        fs, ck = U.forward(gs, alpha=alpha, mu=mu, delta=delta)
        res = U.backward(gs, [cuda(d) for d in dfs], ck, alpha=alpha, mu=mu, delta=delta)
        return ([host(f) for f in fs], host(res["mu"]), float(res["alpha"].item()), host(res["psf"]),
                [host(x) for x in res["g"]])


def _compare(gpu, ref):
    fs, dmu, dal, dpsf, dgs = gpu
    for f, fr in zip(fs, ref["f"]):
        assert rel_err(f, fr) < 1e-5
    assert rel_err(dmu, ref["mu"]) < GRAD_TOL, (dmu, ref["mu"])
    assert abs(dal - ref["alpha"]) <= GRAD_TOL * abs(ref["alpha"]), (dal, ref["alpha"])
    assert rel_err(dpsf, ref["psf"]) < GRAD_TOL
    for dg, dgr in zip(dgs, ref["g"]):
        assert rel_err(dg, dgr) < GRAD_TOL


@pytest.mark.parametrize("sizes,p,L,K,ce", [
    ([32], 5, 1, 4, 2),
    ([32, 24], 5, 2, 6, 4),       # uneven images, ragged last segment
    ([48, 36, 64], 7, 2, 7, 3),   # several tiles per image, ragged segment
    ([72], 9, 3, 5, 5),           # one segment, three levels
    ([96], 3, 1, 3, 1),           # every state checkpointed
    ([28, 32, 42], 5, 2, 4, 2),   # 28 = 2^2 7, 42 = 2 3 7: Bluestein-form transforms beside a 2^a one
])
def test_gradients_match_oracle(mlba, sizes, p, L, K, ce):
    announce(f"unrolled grad vs oracle sizes={sizes} p={p} L={L} K={K} ckpt={ce}")
    H, imgs = _images(sizes, p, 100 + p + K)
    gen = synth.rng(7 + K)
    dfs = [gen.standard_normal((n + p - 1, n + p - 1)) for n in sizes]
    bands = 8 * L + 1
    mu = list(gen.uniform(0.002, 0.02, size=bands))
    alpha, delta = 0.1, 0.3
    gpu = _run(mlba, sizes, p, L, K, ce, H, imgs, dfs, alpha, mu, delta)
    ref = _oracle_sum(H, imgs, dfs, alpha, np.asarray(mu), delta, K, L)
    _compare(gpu, ref)


def test_checkpoint_interval_does_not_change_results(mlba):
    """Recomputed segments are bit-identical to the forward pass, so every
    checkpoint interval gives bit-identical gradients."""
    announce("checkpoint interval invariance")
    sizes, p, L, K = [64, 48], 9, 2, 8
    H, imgs = _images(sizes, p, 55)
    gen = synth.rng(3)
    dfs = [gen.standard_normal((n + p - 1, n + p - 1)) for n in sizes]
    runs = [_run(mlba, sizes, p, L, K, ce, H, imgs, dfs, 0.05, 3e-3, 0.25) for ce in (1, 3, 8)]
    for other in runs[1:]:
        for a, b in zip(runs[0][0], other[0]):
            assert np.array_equal(a, b)
        assert np.array_equal(runs[0][1], other[1])
        assert runs[0][2] == other[2]
        assert np.array_equal(runs[0][3], other[3])
        for a, b in zip(runs[0][4], other[4]):
            assert np.array_equal(a, b)


def test_forward_equals_restore(mlba):
    """The unrolled forward runs the restoration's own tile bodies: f equals
    K iterations of mlba_restore bit for bit."""
    import torch
    announce("unrolled forward == restore")
    sizes, p, L, K = [96, 64], 11, 2, 9
    H, imgs = _images(sizes, p, 77)
    mu = [1e-3 * (1 + b % 4) for b in range(8 * L + 1)]
    with mlba.Unrolled(sizes, p, L, cuda(H), K, 4) as U:
        gs = [cuda(g) for g, _ in imgs]
        fs, _ = U.forward(gs, alpha=0.07, mu=mu, delta=0.3)
        for pl, g, f in zip(U.plans, gs, fs):
            ref, _ = pl.restore(g, alpha=0.07, mu=mu, delta=0.3, iters=K)
            torch.cuda.synchronize()
            assert torch.equal(f, ref)


def test_autograd_function(mlba):
    """loss = ||f - f_true||^2 through torch.autograd: every input gradient
    against the oracle's."""
    import torch
    announce("autograd function")
    n, p, L, K, B = 48, 7, 2, 6, 3
    H, imgs = _images([n] * B, p, 91)
    alpha, delta = 0.08, 0.3
    mu0 = synth.rng(5).uniform(0.002, 0.01, size=8 * L + 1)
    with mlba.Unrolled([n] * B, p, L, cuda(H), K, 2) as U:
        g = torch.stack([cuda(x) for x, _ in imgs]).requires_grad_(True)
        psf = cuda(H).requires_grad_(True)
        a = torch.tensor(alpha, device="cuda", requires_grad=True)
        mu = cuda(mu0).requires_grad_(True)
        truth = torch.stack([cuda(t) for _, t in imgs])
        f = mlba.unrolled_mlba(g, psf, a, mu, U, delta)
        loss = ((f - truth) ** 2).sum()
        loss.backward()
        f_h = host(f.detach())
    dfs = [2.0 * (f_h[i].astype(np.float64) - imgs[i][1]) for i in range(B)]
    ref = _oracle_sum(H, imgs, dfs, alpha, mu0, delta, K, L)
    assert rel_err(host(mu.grad), ref["mu"]) < GRAD_TOL
    assert abs(float(a.grad) - ref["alpha"]) <= GRAD_TOL * abs(ref["alpha"])
    assert rel_err(host(psf.grad), ref["psf"]) < GRAD_TOL
    for i in range(B):
        assert rel_err(host(g.grad[i]), ref["g"][i]) < GRAD_TOL


def test_rejects_unsupported_models(mlba):
    from paper_1504_07234_amd import _lib
    announce("unrolled argument checks")
    H = cuda(synth.gaussian_psf(5, 1.0))
    with pytest.raises(_lib.MLBAError) as e:
        mlba.Unrolled([32], 5, 1, H, 0, 1)
    assert e.value.status == _lib.EINVAL
    with pytest.raises(_lib.MLBAError):
        mlba.Unrolled([32], 5, 1, H, 4, 5)  # ckpt_every > K
    pl = mlba.Plan(32, 5, mlba.REFLECT, mlba.DCT, 1, H)
    import ctypes
    lib = _lib.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 1)(pl._h.value)
    assert lib.mlba_unrolled_create(ctypes.byref(h), 1, arr, 4, 2, None) == _lib.EUNSUPPORTED
    pl.close()


def _oracle_image(args):
    """One image's oracle gradient for loss ||f - f_true||^2, in a pool worker
    (one BLAS thread per worker: several workers with a full thread pool each
    slow each other down by an order of magnitude)."""
    from threadpoolctl import threadpool_limits
    g, H, alpha, mu, delta, K, L, truth = args
    with threadpool_limits(1):
        f, *_ = oadj.unrolled_forward(g, H, alpha, mu, delta, K, L)
        return oadj.unrolled_grad(g, H, alpha, mu, delta, K, L, 2.0 * (f - truth))


def test_full_size_batch_against_oracle(mlba):
    """The benchmarked configuration: 16 images of 256^2, 15x15 Gaussian PSF
    (sigma 2.5), 2 levels (17 thresholds), K = 30, checkpoints every 5, loss
    ||f - f_true||^2.  GPU gradient of the batch vs the sum of the oracle's
    per-image gradients."""
    import torch
    ws = synth.unrolled_workloads()
    w0 = ws[0]
    K, L, ce = w0.iters, w0.levels, w0.extra["ckpt_every"]
    announce(f"full-size unrolled batch {len(ws)}x{w0.n}^2 p={w0.p} K={K} ckpt={ce}")
    gs = [observed(w, oblur)[0] for w in ws]
    delta = omlba.delta_auto(omlba.opnorm(w0.psf, w0.n, 0, 0, w0.alpha0, tol=1e-6))
    mu = np.full(w0.bands, w0.mu)
    with mlba.Unrolled([w.n for w in ws], w0.p, L, cuda(w0.psf), K, ce) as U:
        gd = [cuda(g) for g in gs]
        fs, ck = U.forward(gd, alpha=w0.alpha0, mu=list(mu), delta=delta)
        dfs = [2.0 * (f - cuda(w.truth)) for f, w in zip(fs, ws)]
        res = U.backward(gd, dfs, ck, alpha=w0.alpha0, mu=list(mu), delta=delta)
        torch.cuda.synchronize()
        gpu = {k: host(res[k]) for k in ("mu", "alpha", "psf")}
        dg0 = host(res["g"][0])
    # oracle images in fresh interpreters (never fork a process that holds a HIP context)
    jobs = [(g, w.psf, w.alpha0, mu, delta, K, L, w.truth) for g, w in zip(gs, ws)]
    refs = [None] * len(jobs)
    with cf.ProcessPoolExecutor(max_workers=8, mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(_oracle_image, j): i for i, j in enumerate(jobs)}
        for fut in cf.as_completed(futs):
            refs[futs[fut]] = fut.result()
            announce(f"oracle image {futs[fut]} done")
    ref_mu = sum(r["mu"] for r in refs)
    ref_alpha = sum(r["alpha"] for r in refs)
    ref_psf = sum(r["psf"] for r in refs)
    assert rel_err(gpu["mu"], ref_mu) < GRAD_TOL
    assert abs(float(gpu["alpha"]) - ref_alpha) <= GRAD_TOL * abs(ref_alpha)
    assert rel_err(gpu["psf"], ref_psf) < GRAD_TOL
    assert rel_err(dg0, refs[0]["g"]) < GRAD_TOL
