"""Batched restoration (many uneven images per launch, hipGraph replay).

Each image of a batch runs the same tile bodies as its own plan's
single-image path, so the batched result must equal the per-image result bit
for bit; the per-image path is itself pinned to the FP64 oracle, and one
batch is also compared with the oracle directly.
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import blur as oblur
from oracle import mlba as omlba
from tests._util import announce, cuda, host, max_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


def _problem(n, p, seed, bc=0):
    gen = synth.rng(seed)
    truth = synth.shapes_image(n + p - 1, gen, n_rect=6, n_disk=3, n_bumps=3)
    H = synth.gaussian_psf(p, gen.uniform(1.0, 4.0))
    g = synth.add_noise(oblur.blur(truth, H, 0), synth.white_noise((n, n), gen), gen.uniform(0.005, 0.02))
    return g, H


SIZES = [(64, 9), (96, 13), (128, 25), (192, 11), (256, 17), (72, 5), (384, 21), (144, 15)]


def _make(mlba, specs, levels=2, precond=0, bcs=None):
    plans, gs, Hs = [], [], []
    for i, (n, p) in enumerate(specs):
        bc = 0 if bcs is None else bcs[i]
        g, H = _problem(n, p, 4000 + i)
        plans.append(mlba.Plan(n, p, bc, precond, levels, cuda(H)))
        gs.append(g)
        Hs.append(H)
    return plans, gs, Hs


def test_batched_equals_per_image(mlba):
    import torch
    announce("batched == per-image (eager and graph)")
    plans, gs, _ = _make(mlba, SIZES)
    iters = 15
    alphas = [0.02 + 0.02 * i for i in range(len(plans))]
    deltas = [0.2 + 0.01 * i for i in range(len(plans))]
    mus = [1e-3 * (1 + i % 3) for i in range(len(plans))]
    gdev = [cuda(g) for g in gs]
    ref = []
    for pl, g, a, d, m in zip(plans, gdev, alphas, deltas, mus):
        f, info = pl.restore(g, alpha=a, mu=m, delta=d, iters=iters)
        ref.append((f.clone(), info.rnorm))
    with mlba.Batch(plans, max_iters=iters) as batch:
        for use_graph in (False, True):
            outs, norms = batch.restore(gdev, alpha=alphas, mu=mus, delta=deltas, iters=iters,
                                        use_graph=use_graph, track=True)
            torch.cuda.synchronize()
            for i, (f_ref, rn_ref) in enumerate(ref):
                assert torch.equal(outs[i], f_ref), (use_graph, i)
                assert np.allclose(norms[i], rn_ref, rtol=1e-12, atol=0), (use_graph, i)
    for pl in plans:
        pl.close()


def test_graph_replays_with_eager_work_between(mlba):
    """Every replay of the captured graph equals the eager batched result, with
    unrelated eager GPU work and synchronisations between the replays."""
    import torch
    announce("graph replays")
    plans, gs, _ = _make(mlba, SIZES[:5])
    iters = 10
    gdev = [cuda(g) for g in gs]
    with mlba.Batch(plans, max_iters=iters) as batch:
        eager, _ = batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.25, iters=iters, use_graph=False)
        eager = [e.clone() for e in eager]
        for rep in range(4):
            junk = torch.randn(1 << 20, device="cuda").cumsum(0)
            _ = plans[0].apply_A(torch.rand(plans[0].N, plans[0].N, device="cuda"))
            torch.cuda.synchronize()
            outs, _ = batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.25, iters=iters, use_graph=True)
            torch.cuda.synchronize()
            for i in range(len(plans)):
                assert torch.equal(outs[i], eager[i]), (rep, i)
            del junk
    for pl in plans:
        pl.close()


def test_batched_reflective_dct(mlba):
    import torch
    announce("batched reflective + DCT")
    specs = [(64, 9), (96, 7), (128, 15), (192, 9)]
    plans, gs, _ = _make(mlba, specs, levels=3, precond=1, bcs=[1, 0, 1, 3])
    iters = 12
    gdev = [cuda(g) for g in gs]
    ref = [pl.restore(g, alpha=0.1, mu=2e-3, delta=0.3, iters=iters)[0].clone() for pl, g in zip(plans, gdev)]
    with mlba.Batch(plans, max_iters=iters) as batch:
        outs, _ = batch.restore(gdev, alpha=0.1, mu=2e-3, delta=0.3, iters=iters, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(outs[i], ref[i]), i
    for pl in plans:
        pl.close()


def test_batched_antireflective(mlba):
    """Antireflective images (pad in A, reblur in place of A^T) batched with
    rectangular and periodic ones, BCCB preconditioner: equal to the per-image
    path bit for bit, and one image against the FP64 oracle."""
    import torch
    announce("batched antireflective + BCCB")
    specs = [(64, 9), (96, 7), (128, 15), (96, 11)]
    bcs = [4, 0, 4, 2]
    plans, gs, Hs = _make(mlba, specs, levels=2, precond=0, bcs=bcs)
    iters = 12
    gdev = [cuda(g) for g in gs]
    ref = [pl.restore(g, alpha=0.2, mu=2e-3, delta=0.1, iters=iters)[0].clone() for pl, g in zip(plans, gdev)]
    with mlba.Batch(plans, max_iters=iters) as batch:
        outs, _ = batch.restore(gdev, alpha=0.2, mu=2e-3, delta=0.1, iters=iters, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(outs[i], ref[i]), i
        got = host(outs[2])
    n, p = specs[2]
    want = omlba.mlba(gs[2], Hs[2], oblur.ANTIREFLECT, 0, 2, np.full(iters, 0.2), np.full(iters + 1, 0.1), 2e-3,
                      iters)["f"]
    assert rel_err(got, want) < 1e-4
    for pl in plans:
        pl.close()


def test_batched_against_oracle(mlba):
    announce("batched vs FP64 oracle")
    specs = [(64, 9), (96, 17), (192, 11)]
    plans, gs, Hs = _make(mlba, specs)
    iters = 30
    alphas = [0.05, 0.1, 0.03]
    deltas = [omlba.delta_auto(omlba.opnorm(H, n, 0, 0, a, tol=1e-6)) for (n, p), H, a in zip(specs, Hs, alphas)]
    with mlba.Batch(plans, max_iters=iters) as batch:
        outs, norms = batch.restore([cuda(g) for g in gs], alpha=alphas, mu=1e-3, delta=deltas, iters=iters,
                                    use_graph=True, track=True)
        outs = [host(o) for o in outs]
    for i, ((n, p), H, g) in enumerate(zip(specs, Hs, gs)):
        ref = omlba.mlba(g, H, 0, 0, 2, np.full(iters, alphas[i]), np.full(iters + 1, deltas[i]), 1e-3, iters)
        assert rel_err(outs[i], ref["f"]) < 1e-4
        assert rel_err(norms[i], ref["rnorm"]) < 1e-4
    for pl in plans:
        pl.close()


def test_batched_resume_state(mlba):
    """Caller-owned states: 4 + 6 batched iterations equal 10."""
    import torch
    announce("batched resume")
    plans, gs, _ = _make(mlba, SIZES[:3])
    gdev = [cuda(g) for g in gs]
    with mlba.Batch(plans, max_iters=10) as batch:
        full, _ = batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.3, iters=10, use_graph=False)
        full = [f.clone() for f in full]
        zs = [torch.zeros(p.bands, p.N, p.N, device="cuda") for p in plans]
        batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.3, iters=4, zs=zs, use_graph=True)
        outs, _ = batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.3, iters=6, zs=zs, use_graph=True)
        torch.cuda.synchronize()
        for i in range(3):
            assert torch.equal(outs[i], full[i])
    for pl in plans:
        pl.close()


def test_batch_rejects_mixed_levels(mlba):
    from paper_1504_07234_amd import _lib
    announce("batch argument checks")
    a = mlba.Plan(64, 9, 0, 0, 2, cuda(synth.gaussian_psf(9, 2.0)))
    b = mlba.Plan(64, 9, 0, 0, 3, cuda(synth.gaussian_psf(9, 2.0)))
    lib = _lib.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 2)(a._h.value, b._h.value)
    assert lib.mlba_batch_create(ctypes.byref(h), 2, arr, 10, None) == _lib.EINVAL
    arr = (ctypes.c_void_p * 2)(a._h.value, a._h.value)
    assert lib.mlba_batch_create(ctypes.byref(h), 2, arr, 10, None) == _lib.EINVAL
    a.close()
    b.close()


def test_tile_choices_do_not_change_results(mlba):
    """Every tile shape the autotuner can pick computes each output with the
    same arithmetic: results are bit-identical across choices, including the
    autotuner's own pick (graph re-captured after each change)."""
    import torch
    announce("batched tile choices bitwise")
    plans, gs, _ = _make(mlba, SIZES)
    iters = 6
    gdev = [cuda(g) for g in gs]
    with mlba.Batch(plans, max_iters=iters) as batch:
        ref, _ = batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.25, iters=iters, use_graph=True)
        ref = [r.clone() for r in ref]
        choices = [((2, 1), 0, 0), ((1, 2), 0, 0), ((2, 2), 0, 0)]
        choices += [((1, 1), c, 0) for c in (1, 2, 4)]
        choices += [((1, 1), 0, c) for c in (1, 2, 4, 8, 16)]
        for conv_rows, rc, cc in choices:
            batch.set_tiles(conv_rows, rc, cc)
            outs, _ = batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.25, iters=iters, use_graph=True)
            torch.cuda.synchronize()
            for i in range(len(plans)):
                assert torch.equal(outs[i], ref[i]), (conv_rows, rc, cc, i)
        tuned = batch.autotune(reps=2)
        assert tuned["conv_rows"][0] in (1, 2) and tuned["conv_rows"][1] in (1, 2)
        assert all(t > 0 for t in tuned["rows_ms"] + tuned["cols_ms"])
        outs, _ = batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.25, iters=iters, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(outs[i], ref[i]), ("tuned", i)
    for pl in plans:
        pl.close()


@pytest.mark.parametrize("precond", [0, 3])
def test_batched_bluestein_sizes(mlba, precond):
    """Images whose transform lengths have a prime factor >= 7 (196 = 2^2 7^2
    and 70 = 2 * 5 * 7 for the BCCB preconditioner; the antireflective
    transform lengths 390 and 140 of 196 and 71) batched with 5-smooth ones:
    equal to the per-image path bit for bit, and one against the oracle."""
    import torch
    announce(f"batched Bluestein sizes precond={precond}")
    specs = [(196, 11), (70, 9), (128, 15)] if precond == 0 else [(196, 9), (71, 7), (65, 9)]
    bcs = None if precond == 0 else [4, 4, 4]
    plans, gs, Hs = _make(mlba, specs, levels=2, precond=precond, bcs=bcs)
    iters = 10
    alpha, mu, delta = (0.05, 1e-3, 0.2) if precond == 0 else (0.05, 1e-3, 0.1)
    gdev = [cuda(g) for g in gs]
    ref = [pl.restore(g, alpha=alpha, mu=mu, delta=delta, iters=iters)[0].clone() for pl, g in zip(plans, gdev)]
    with mlba.Batch(plans, max_iters=iters) as batch:
        outs, _ = batch.restore(gdev, alpha=alpha, mu=mu, delta=delta, iters=iters, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(outs[i], ref[i]), i
        got = host(outs[0])
    bc = oblur.RECT if precond == 0 else oblur.ANTIREFLECT
    want = omlba.mlba(gs[0], Hs[0], bc, precond, 2, np.full(iters, alpha), np.full(iters + 1, delta), mu,
                      iters)["f"]
    print(f"  image 0 vs oracle {rel_err(got, want):.2e}", flush=True)
    assert rel_err(got, want) < 1e-4
    for pl in plans:
        pl.close()


@pytest.mark.parametrize("levels,precond,bcs", [(2, 0, None), (3, 0, [0, 3, 2, 4, 0, 0, 3, 0]),
                                                (3, 1, [1, 0, 1, 3, 1, 0, 1, 3]), (1, 0, None)])
def test_batched_implicit_equals_per_image(mlba, levels, precond, bcs):
    """The implicit state (omega, z = W omega; the low-pass chain, the
    shrink-synthesis levels and omega += A^T t in the A^T launch) batched over
    uneven images equals per-image implicit restorations bit for bit, eager and
    from the graph, with the residual-norm histories."""
    import torch
    announce(f"batched implicit == per-image implicit (levels={levels}, precond={precond})")
    specs = SIZES if precond == 0 else [(64, 9), (96, 7), (128, 15), (192, 9), (72, 5), (160, 13), (96, 11), (64, 3)]
    plans, gs, _ = _make(mlba, specs, levels=levels, precond=precond, bcs=bcs)
    iters = 12
    alphas = [0.03 + 0.02 * i for i in range(len(plans))]
    deltas = [0.15 + 0.01 * i for i in range(len(plans))]
    mus = [1e-3 * (1 + i % 3) for i in range(len(plans))]
    gdev = [cuda(g) for g in gs]
    ref = []
    for pl, g, a, d, m in zip(plans, gdev, alphas, deltas, mus):
        f, info = pl.restore(g, alpha=a, mu=m, delta=d, iters=iters, implicit=True)
        ref.append((f.clone(), info.rnorm))
    with mlba.Batch(plans, max_iters=iters) as batch:
        for use_graph in (False, True, True):
            outs, norms = batch.restore(gdev, alpha=alphas, mu=mus, delta=deltas, iters=iters, use_graph=use_graph,
                                        track=True, implicit=True)
            torch.cuda.synchronize()
            for i, (f_ref, rn_ref) in enumerate(ref):
                assert torch.equal(outs[i], f_ref), (use_graph, i)
                assert np.allclose(norms[i], rn_ref, rtol=1e-12, atol=0), (use_graph, i)
        # the explicit state again on the same batch (descriptors and graph switch back)
        eo, _ = batch.restore(gdev, alpha=alphas, mu=mus, delta=deltas, iters=iters, use_graph=True)
        for i, (pl, g, a, d, m) in enumerate(zip(plans, gdev, alphas, deltas, mus)):
            fe, _ = pl.restore(g, alpha=a, mu=m, delta=d, iters=iters)
            assert torch.equal(eo[i], fe), ("explicit after implicit", i)
    for pl in plans:
        pl.close()


def test_batched_implicit_against_oracle_and_resume(mlba):
    """Batched implicit restorations against the FP64 oracle (1e-4, image and
    residual norms, element-wise bar too), and caller-owned omega states: 5 + 7
    iterations equal 12."""
    import torch
    announce("batched implicit vs FP64 oracle, resume")
    specs = [(64, 9), (96, 17), (192, 11), (128, 25)]
    plans, gs, Hs = _make(mlba, specs)
    iters = 30
    alphas = [0.05, 0.1, 0.03, 0.08]
    deltas = [omlba.delta_auto(omlba.opnorm(H, n, 0, 0, a)) for (n, p), H, a in zip(specs, Hs, alphas)]
    gdev = [cuda(g) for g in gs]
    with mlba.Batch(plans, max_iters=iters) as batch:
        outs, norms = batch.restore(gdev, alpha=alphas, mu=1e-3, delta=deltas, iters=iters, use_graph=True,
                                    track=True, implicit=True)
        got = [host(o) for o in outs]
        full, _ = batch.restore(gdev, alpha=alphas, mu=1e-3, delta=deltas, iters=12, use_graph=False, implicit=True)
        full = [f.clone() for f in full]
        zs = [torch.zeros(p.N, p.N, device="cuda") for p in plans]
        batch.restore(gdev, alpha=alphas, mu=1e-3, delta=deltas, iters=5, zs=zs, use_graph=True, implicit=True)
        res, _ = batch.restore(gdev, alpha=alphas, mu=1e-3, delta=deltas, iters=7, zs=zs, use_graph=True,
                               implicit=True)
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(res[i], full[i]), i
    for i, ((n, p), H, g) in enumerate(zip(specs, Hs, gs)):
        ref = omlba.mlba(g, H, 0, 0, 2, np.full(iters, alphas[i]), np.full(iters + 1, deltas[i]), 1e-3, iters)
        print(f"  image {i}: rel {rel_err(got[i], ref['f']):.2e} max {max_err(got[i], ref['f']):.2e}", flush=True)
        assert rel_err(got[i], ref["f"]) < 1e-4 and max_err(got[i], ref["f"]) < 1e-4
        assert rel_err(norms[i], ref["rnorm"]) < 1e-4
    for pl in plans:
        pl.close()


def test_tile_changes_allocate_nothing(mlba):
    """The tile maps are sized at creation for the choice with the most
    workgroups: set_tiles and the autotuner leave the device's free memory
    unchanged."""
    import torch
    announce("batch tile changes allocate nothing")
    plans, gs, _ = _make(mlba, SIZES[:4])
    gdev = [cuda(g) for g in gs]
    with mlba.Batch(plans, max_iters=4) as batch:
        batch.restore(gdev, alpha=0.05, mu=1e-3, delta=0.25, iters=4, use_graph=False)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for conv_rows, rc, cc in (((2, 2), 1, 1), ((1, 1), 4, 16), ((1, 2), 0, 0)):
            batch.set_tiles(conv_rows, rc, cc)
        batch.autotune(reps=1)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
    for pl in plans:
        pl.close()
