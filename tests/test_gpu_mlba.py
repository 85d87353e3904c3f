"""End-to-end parity of the HIP restoration loop (eq. MLBA2) against the FP64
oracle, on the seeded workloads, through the C ABI ``mlba_restore``.

Bar: the restored image after the full iteration count within 1e-4
(||.||_2-relative, and element by element relative to the image's largest
value) of the oracle, the residual-norm history within 1e-4.  The workload
runs take their alpha_k and delta_k from the library's own schedules (the
geometric alpha_k and the automatic step of section 3's convergence theorem,
with the norm by Lanczos on the GPU) and compare them with the oracle's
tables; the other runs feed both sides the oracle's tables.
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import blur as oblur
from oracle import mlba as omlba
from tests._util import announce, cached, cuda, host, max_err, observed, rel_err, workload_key

pytestmark = pytest.mark.gpu

TOL_IMAGE = 1e-4
TOL_MAX = 1e-4     # max |f - f_ref| / max |f_ref|
# the automatic step against the oracle's: the norm comes from FP32 applications
# of A, P and A^T (Lanczos on the GPU, ARPACK in FP64 in the oracle), so it
# takes the per-operator bar
TOL_DELTA = 1e-5


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


def _schedules(w, iters):
    def compute():
        alphas = omlba.alpha_table(w.alpha_kind, w.alpha0, iters, w.alpha_ratio, w.alpha_floor)
        return alphas, omlba.delta_table(w.psf, w.n, w.bc, w.precond, alphas, w.delta, iters + 1)
    return cached(("schedules",) + workload_key(w, iters), compute)


def _run_both(mlba, w, iters, alphas, deltas, g):
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        f, info = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=iters)
        f = host(f)
    ref = omlba.mlba(g, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, iters)
    return f, info, ref


def _run_library_schedules(mlba, w, iters, g, **kw):
    """The GPU with the library's own alpha_k / delta_k (no tables); the oracle
    with its alpha_table / delta_table for the same workload parameters."""
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        f, info = plan.restore(cuda(g), alpha=w.alpha0, alpha_kind=w.alpha_kind, alpha_ratio=w.alpha_ratio,
                               alpha_floor=w.alpha_floor, mu=w.mu, delta=w.delta, iters=iters, **kw)
        f = host(f)
    alphas, deltas = _schedules(w, iters)
    ref = cached(("mlba",) + workload_key(w, iters),
                 lambda: omlba.mlba(g, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, iters))
    return f, info, ref, alphas, deltas


def _check_schedules(info, alphas, deltas):
    ea = np.max(np.abs(np.asarray(info.alphas) / alphas - 1.0))
    rd = np.abs(np.asarray(info.deltas) / deltas - 1.0)
    ed, kd = np.max(rd), int(np.argmax(rd))
    print(f"  alpha_k rel err {ea:.1e}, delta_k rel err {ed:.1e} at k = {kd} (alpha {alphas[min(kd, len(alphas) - 1)]:.5f}, "
          f"delta {deltas[kd]:.9f}); distinct delta_k {len(set(info.deltas))}", flush=True)
    assert len(info.alphas) == len(alphas) and len(info.deltas) == len(deltas)
    assert ea <= 1e-14
    assert ed <= TOL_DELTA


def test_small_workload_auto_step(mlba):
    """72 x 72 unknown, 9 x 9 Gaussian, BCCB alpha = 0.05, 1 level, 50 its, the
    library's automatic step (the workload's literal unit step diverges)."""
    w = dataclasses.replace(synth.make_workload("plain-fp64-72"), delta=0.0)
    announce("restore plain-fp64-72 auto step (library schedule)")
    g, nn = observed(w, oblur)
    f, info, ref, alphas, deltas = _run_library_schedules(mlba, w, w.iters, g)
    assert info.status == 0 and info.iters_done == w.iters
    _check_schedules(info, alphas, deltas)
    e, em = rel_err(f, ref["f"]), max_err(f, ref["f"])
    print(f"  image rel err {e:.2e} max {em:.2e}; rnorm last gpu {info.rnorm[-1]:.5f} "
          f"oracle {ref['rnorm'][-1]:.5f}", flush=True)
    assert e < TOL_IMAGE and em < TOL_MAX
    assert rel_err(info.rnorm, ref["rnorm"]) < TOL_IMAGE


def test_small_workload_literal_step_diverges(mlba):
    """The literal unit step violates the convergence condition (the operator
    norm is about 3.2 at alpha = 0.05): both sides diverge and the library
    reports MLBA_WARN_DIVERGED."""
    w = synth.make_workload("plain-fp64-72")
    announce("restore plain-fp64-72 literal step")
    g, _ = observed(w, oblur)
    alphas = np.full(w.iters, w.alpha0)
    deltas = np.full(w.iters + 1, 1.0)
    f, info, ref = _run_both(mlba, w, w.iters, alphas, deltas, g)
    assert info.status == 1  # MLBA_WARN_DIVERGED
    assert ref["rnorm"][-1] > 1e3 * ref["rnorm"][0]
    # both blow up along the same direction: the FP32 history still tracks FP64
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-3


@pytest.mark.parametrize("name", ["rect-bccb-512", "reflect-dct-512", "rect-bccb-geometric-512"])
def test_512_workloads_200_iterations(mlba, name):
    """The three 512 workloads with the library's schedules: constant alpha with
    the automatic step (BCCB and DCT), and the geometric alpha_k (no table) with
    one automatic step per distinct alpha_k."""
    w = synth.make_workload(name)
    announce(f"restore {name} {w.iters} iterations (library schedule)")
    g, nn = observed(w, oblur)
    f, info, ref, alphas, deltas = _run_library_schedules(mlba, w, w.iters, g)
    _check_schedules(info, alphas, deltas)
    e, em = rel_err(f, ref["f"]), max_err(f, ref["f"])
    er = rel_err(info.rnorm, ref["rnorm"])
    print(f"  image rel err {e:.2e} max {em:.2e}, rnorm rel err {er:.2e}, final rnorm {info.rnorm[-1]:.4f} "
          f"(noise {nn:.4f})", flush=True)
    assert info.status == 0 and info.iters_done == w.iters
    assert e < TOL_IMAGE and em < TOL_MAX
    assert er < TOL_IMAGE


def test_table_schedules_512(mlba):
    """The table path (MLBA_ALPHA_TABLE and delta_table) on the geometric 512
    workload, fed the oracle's tables."""
    w = synth.make_workload("rect-bccb-geometric-512")
    iters = 60
    announce(f"restore rect-bccb-geometric-512 {iters} iterations (oracle tables)")
    g, nn = observed(w, oblur)
    alphas, deltas = _schedules(w, iters)
    f, info, ref = _run_both(mlba, w, iters, alphas, deltas, g)
    assert np.array_equal(info.alphas, alphas) and np.array_equal(info.deltas, deltas)
    e, em = rel_err(f, ref["f"]), max_err(f, ref["f"])
    print(f"  image rel err {e:.2e} max {em:.2e}", flush=True)
    assert e < TOL_IMAGE and em < TOL_MAX
    assert rel_err(info.rnorm, ref["rnorm"]) < TOL_IMAGE


def test_short_delta_table_rejected(mlba):
    """delta_table needs k0 + iters + 1 values (the last one scales the
    returned image); a shorter table is MLBA_EINVAL, not a read past its end."""
    from paper_1504_07234_amd import _lib
    w = synth.make_workload("plain-fp64-72")
    announce("short delta table")
    g, _ = observed(w, oblur)
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        for k0, n_tab in ((0, 10), (3, 13)):
            with pytest.raises(_lib.MLBAError) as ei:
                plan.restore(cuda(g), alpha=0.05, mu=w.mu, delta_table=np.full(n_tab, 0.2), iters=10, k0=k0)
            assert ei.value.status == _lib.EINVAL
        _, info = plan.restore(cuda(g), alpha=0.05, mu=w.mu, delta_table=np.full(11, 0.2), iters=10)
        assert info.status == 0 and info.deltas == [0.2] * 11


def test_full_size_iterations(mlba):
    """2048 x 2048 observed, 31 x 31 disk, 3 levels: the bench workload, a few
    iterations compared in full (state z and image), with the direct blur and
    with the FFT blur (whose residual and A^T row passes run fused with the
    preconditioner's row passes), in both states."""
    w = synth.make_workload("rect-bccb-2048")
    iters = 3
    announce(f"restore rect-bccb-2048 {iters} iterations")
    g, _ = observed(w, oblur)
    alphas = np.full(iters, w.alpha0)
    deltas = np.full(iters + 1, 0.3)
    ref = omlba.mlba(g, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, iters)
    import torch
    for blur, implicit in ((mlba.BLUR_DIRECT, False), (mlba.BLUR_FFT, False), (mlba.BLUR_FFT, True)):
        announce(f"  blur={'fft' if blur == mlba.BLUR_FFT else 'direct'} implicit={implicit}")
        with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
            plan.set_blur(blur)
            shape = (plan.N, plan.N) if implicit else (plan.bands, plan.N, plan.N)
            z = torch.zeros(shape, dtype=torch.float32, device="cuda")
            f, info = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=iters, z=z,
                                   implicit=implicit)
            if implicit:
                z = plan.analysis(z)  # z = W omega
            f, z = host(f), host(z)
        print(f"  image {rel_err(f, ref['f']):.2e} state {rel_err(z, ref['z']):.2e} "
              f"rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
        assert rel_err(f, ref["f"]) < 1e-5
        assert rel_err(z, ref["z"]) < 1e-5
        assert rel_err(info.rnorm, ref["rnorm"]) < 1e-6


@pytest.mark.parametrize("bc,pc", [(oblur.ZERO, 0), (oblur.REFLECT, 0), (oblur.REFLECT, 1), (oblur.PERIODIC, 0)])
def test_full_size_square_models(mlba, bc, pc):
    """The bench's square-model runs at full size: 2048 x 2048 image, 31 x 31
    disk, 3 levels, implicit state, FFT-grid blur (the pad on the grid and E^T
    folded back; periodic + BCCB: the residual in the spectrum), 3 iterations
    against the oracle, image and residual norms element by element."""
    w = synth.make_workload("rect-bccb-2048")
    iters, n = 3, w.n
    announce(f"restore 2048 bc={bc} precond={pc} {iters} iterations, FFT blur, implicit")
    g, _ = observed(w, oblur)
    alphas = np.full(iters, w.alpha0)
    deltas = np.full(iters + 1, 0.3)
    ref = omlba.mlba(g, w.psf, bc, pc, w.levels, alphas, deltas, w.mu, iters)
    with mlba.Plan(n, w.p, bc, pc, w.levels, cuda(w.psf)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        plan.profile_begin(iters)
        f, info = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=iters, implicit=True)
        plan.profile_end()
        kern = plan.profile_kernels()
        f = host(f)
    e, em, er = rel_err(f, ref["f"]), max_err(f, ref["f"]), rel_err(info.rnorm, ref["rnorm"])
    print(f"  image {e:.2e} max {em:.2e} rnorm {er:.2e}", flush=True)
    assert e < 1e-5 and em < 1e-4
    assert er < 1e-6
    spectral = bc == oblur.PERIODIC and pc == 0
    assert ("fc_cols" in kern) == (not spectral)


@pytest.mark.parametrize("n,p,bc,pc,L", [(96, 17, 0, 0, 2), (96, 17, 1, 1, 3), (192, 11, 3, 0, 2),
                                         (128, 7, 2, 0, 4), (384, 25, 0, 1, 2)])
def test_ragged_and_mixed_models(mlba, n, p, bc, pc, L):
    announce(f"restore n={n} p={p} bc={bc} pc={pc} L={L}")
    gen = synth.rng(n + p + bc * 7 + pc)
    truth = synth.shapes_image(n + p - 1, gen, n_rect=6, n_disk=3, n_bumps=3)
    H = synth.motion_psf(p, p - 2.0, gen.uniform(0, np.pi))
    b = oblur.blur(truth, H, 0)
    g = synth.add_noise(b, synth.white_noise((n, n), gen), 0.01)
    iters = 40
    alphas = np.full(iters, 0.1)
    d = omlba.delta_auto(omlba.opnorm(H, n, bc, pc, 0.1, tol=1e-6))
    deltas = np.full(iters + 1, d)
    mu = np.linspace(1e-3, 3e-3, 8 * L + 1)
    with mlba.Plan(n, p, bc, pc, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha_table=alphas, mu=mu, delta_table=deltas, iters=iters)
        f = host(f)
    ref = omlba.mlba(g, H, bc, pc, L, alphas, deltas, mu, iters)
    assert rel_err(f, ref["f"]) < TOL_IMAGE and max_err(f, ref["f"]) < TOL_MAX
    assert rel_err(info.rnorm, ref["rnorm"]) < TOL_IMAGE


def test_resume_and_determinism(mlba):
    import torch
    w = synth.make_workload("plain-fp64-72")
    announce("resume + determinism")
    g, _ = observed(w, oblur)
    it = 12
    alphas = np.full(it, 0.05)
    deltas = np.full(it + 1, 0.25)
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        z1 = torch.zeros((plan.bands, plan.N, plan.N), device="cuda")
        f1, i1 = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=it, z=z1)
        z2 = torch.zeros_like(z1)
        _, ia = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=5, z=z2)
        f2, ib = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=7, k0=5, z=z2)
        f3, i3 = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=it)
        assert torch.equal(z1, z2)
        assert torch.equal(f1, f2) and torch.equal(f1, f3)
        assert i1.rnorm == ia.rnorm + ib.rnorm == i3.rnorm


@pytest.mark.parametrize("fft_blur", [False, True])
def test_discrepancy_stop(mlba, fft_blur):
    """eq. (discrpr): stop at the first k with ||r^k|| <= gamma * ||eta||; with
    the FFT blur the residual norm is summed by the preconditioner's column
    pass before the check."""
    w = synth.make_workload("plain-fp64-72")
    announce(f"discrepancy stop fft_blur={fft_blur}")
    g, nn = observed(w, oblur)
    it = 50
    alphas = np.full(it, 0.05)
    d = omlba.delta_auto(omlba.opnorm(w.psf, w.n, 0, 0, 0.05))
    deltas = np.full(it + 1, d)
    ref = omlba.mlba(g, w.psf, 0, 0, 1, alphas, deltas, w.mu, it)
    gamma = 1.2
    k_star = int(np.argmax(ref["rnorm"] <= gamma * nn))
    assert ref["rnorm"][k_star] <= gamma * nn and k_star > 0
    with mlba.Plan(w.n, w.p, 0, 0, 1, cuda(w.psf)) as plan:
        if fft_blur:
            plan.set_blur(mlba.BLUR_FFT)
        f, info = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=it,
                               stop=(nn, gamma, 1))
        f = host(f)
    assert info.iters_done == k_star
    ref_k = omlba.mlba(g, w.psf, 0, 0, 1, alphas, deltas, w.mu, k_star)
    assert rel_err(f, ref_k["f"]) < TOL_IMAGE and max_err(f, ref_k["f"]) < TOL_MAX
