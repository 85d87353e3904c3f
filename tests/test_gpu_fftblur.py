"""The blur A and its transpose computed by FFTs of an M x M grid (section
2.1): the rectangular model's unknown, or a square model's image with its pad
of Table 1 (zero, reflective, periodic) placed on the grid and the transpose
folded back by E^T; against the FP64 oracle, and the restoration with it.
Bars: 1e-5 (relative, L2) and 1e-4 (element by element, relative to the
largest value) per operator, 1e-4 on restored images."""
import numpy as np
import pytest

import synth
from oracle import blur as ob
from oracle import alg4 as oa
from oracle import mlba as omlba
from tests._util import announce, cuda, host, max_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


# (n, p): ragged grids, odd N, the largest PSF, the compiled 1152 grid, the
# 3072-point limit, the bench shape (the compiled 2304 grid)
CASES = [(8, 1), (64, 9), (100, 17), (97, 5), (256, 49), (1000, 49), (2048, 31), (3000, 49)]


@pytest.mark.parametrize("n,p", CASES)
def test_fft_blur_and_transpose(mlba, n, p):
    announce(f"FFT blur n={n} p={p}")
    g = synth.rng(9000 + n + p)
    H = g.random((p, p)) + 0.05
    H /= H.sum()
    N = n + p - 1
    u = g.standard_normal((N, N))
    y = g.standard_normal((n, n))
    gobs = g.standard_normal((n, n))
    with mlba.Plan(n, p, mlba.RECT, mlba.NONE, 1, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        Au = host(plan.apply_A(cuda(u)))
        Aty = host(plan.apply_At(cuda(y)))
        res = host(plan.residual(cuda(gobs), cuda(u)))
    ref_A = ob.blur(u, H, ob.RECT)
    ref_At = ob.blurT(y, H, ob.RECT)
    print(f"  A {rel_err(Au, ref_A):.2e}  A^T {rel_err(Aty, ref_At):.2e}", flush=True)
    assert rel_err(Au, ref_A) < 1e-5 and max_err(Au, ref_A) < 1e-4
    assert rel_err(Aty, ref_At) < 1e-5 and max_err(Aty, ref_At) < 1e-4
    assert rel_err(res, gobs - ref_A) < 1e-5


# square models: (n, p) with p = 1 (no pad), odd n, pads wider than a row
# pair, the largest PSF, the bench size
SQUARE = [(8, 1), (64, 9), (97, 5), (100, 17), (256, 49), (2048, 31)]


@pytest.mark.parametrize("bc", ["REFLECT", "PERIODIC", "ZERO"])
@pytest.mark.parametrize("n,p", SQUARE)
def test_fft_blur_square_models(mlba, bc, n, p):
    announce(f"FFT blur {bc} n={n} p={p}")
    g = synth.rng(9100 + n + p)
    H = g.random((p, p)) + 0.05
    H /= H.sum()
    u = g.standard_normal((n, n))
    y = g.standard_normal((n, n))
    gobs = g.standard_normal((n, n))
    obc = getattr(ob, bc)
    with mlba.Plan(n, p, getattr(mlba, bc), mlba.NONE, 1, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        Au = host(plan.apply_A(cuda(u)))
        Aty = host(plan.apply_At(cuda(y)))
        res = host(plan.residual(cuda(gobs), cuda(u)))
        plan.set_blur(mlba.BLUR_DIRECT)
        Aty_d = host(plan.apply_At(cuda(y)))
    ref_A = ob.blur(u, H, obc)
    ref_At = ob.blurT(y, H, obc)
    print(f"  A {rel_err(Au, ref_A):.2e} max {max_err(Au, ref_A):.2e}  A^T {rel_err(Aty, ref_At):.2e} "
          f"max {max_err(Aty, ref_At):.2e}", flush=True)
    assert rel_err(Au, ref_A) < 1e-5 and max_err(Au, ref_A) < 1e-4
    assert rel_err(Aty, ref_At) < 1e-5 and max_err(Aty, ref_At) < 1e-4
    assert rel_err(res, gobs - ref_A) < 1e-5
    assert rel_err(Aty, Aty_d) < 1e-5


def test_fft_blur_fits(mlba):
    from paper_1504_07234_amd import _lib
    announce("FFT blur argument checks")
    H = cuda(synth.gaussian_psf(5, 1.0))
    with mlba.Plan(3100, 5, mlba.RECT, mlba.NONE, 1, H) as plan:  # M would exceed 3072
        with pytest.raises(_lib.MLBAError) as e:
            plan.set_blur(mlba.BLUR_FFT)
        assert e.value.status == _lib.EUNSUPPORTED
        assert plan.autotune(reps=1)["fft_ms"] is None


@pytest.mark.parametrize("implicit", [False, True])
def test_restore_with_fft_blur(mlba, implicit):
    """A 512 workload restored with the FFT blur: same oracle bar as the direct blur."""
    w = synth.make_workload("rect-bccb-512")
    announce(f"restore rect-bccb-512 with FFT blur implicit={implicit}")
    g = synth.add_noise(ob.blur(w.truth, w.psf, ob.RECT), w.xi, w.noise_level)
    iters = 60
    alphas = np.full(iters, w.alpha0)
    deltas = omlba.delta_table(w.psf, w.n, w.bc, w.precond, alphas, 0.0, iters + 1)
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        f, info = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=iters,
                               implicit=implicit)
        f = host(f)
        # and the direct blur on the same plan agrees
        plan.set_blur(mlba.BLUR_DIRECT)
        f2, _ = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=iters,
                             implicit=implicit)
        f2 = host(f2)
    ref = omlba.mlba(g, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, iters)
    print(f"  fft {rel_err(f, ref['f']):.2e} direct {rel_err(f2, ref['f']):.2e}", flush=True)
    assert rel_err(f, ref["f"]) < 1e-4 and max_err(f, ref["f"]) < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4
    assert rel_err(f, f2) < 1e-4


def test_autotune_picks_a_working_blur(mlba):
    w = synth.make_workload("rect-bccb-2048")
    announce("plan autotune at 2048, p = 31")
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        t = plan.autotune(reps=3)
        print(f"  {t}", flush=True)
        assert t["blur"] in ("fft", "direct") and t["fft_ms"] is not None
        u = synth.rng(3).standard_normal((plan.N, plan.N))
        assert rel_err(host(plan.apply_A(cuda(u))), ob.blur(u, w.psf, ob.RECT)) < 1e-5


@pytest.mark.parametrize("n,p,pc,implicit", [(97, 9, 2, False), (96, 9, 1, True), (96, 9, 0, True),
                                             (96, 9, 0, False)])
def test_restore_small_fft_blur_and_kernel_profile(mlba, n, p, pc, implicit):
    """Without a spectral preconditioner (P = I) the FFT blur runs its three
    passes; with the BCCB matrix or the DCT of Algorithm 3 the residual row
    pass is fused with the preconditioner's forward row pass and the
    preconditioner's inverse row pass with the forward row pass of A^T.  Both
    against the oracle, and the kernel profile of the iteration."""
    announce(f"restore n={n} p={p} precond={pc} FFT blur implicit={implicit}")
    gen = synth.rng(4400 + n + pc)
    H = synth.gaussian_psf(p, 1.5)
    N = n + p - 1
    truth = synth.shapes_image(N, gen, n_rect=6, n_disk=3)
    b = ob.blur(truth, H, ob.RECT)
    g = synth.add_noise(b, synth.white_noise((n, n), gen), 0.01)
    iters = 25
    alphas = np.full(iters + 1, 0.05)
    deltas = omlba.delta_table(H, n, ob.RECT, pc, alphas, 0.0, iters + 1)
    with mlba.Plan(n, p, mlba.RECT, pc, 2, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        plan.profile_begin(iters)
        f, info = plan.restore(cuda(g), alpha_table=alphas[:iters], mu=1e-3, delta_table=deltas, iters=iters,
                               implicit=implicit)
        phases, rec = plan.profile_end()
        kern = plan.profile_kernels()
        f = host(f)
    ref = omlba.mlba(g, H, ob.RECT, pc, 2, alphas[:iters], deltas, 1e-3, iters)
    print(f"  image {rel_err(f, ref['f']):.2e} rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
    assert rel_err(f, ref["f"]) < 1e-4 and max_err(f, ref["f"]) < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4
    assert rec == iters
    fused = pc in (0, 1)  # BCCB and DCT: P's row passes run inside the grid's
    assert kern["fc_cols"][1] == 2 * iters
    assert kern.get("fc_residual_precond_rows", (0, 0))[1] == (iters if fused else 0)
    assert kern.get("precond_rows_fc_fwd", (0, 0))[1] == (iters if fused else 0)
    assert kern.get("fc_rows_fwd", (0, 0))[1] == (1 if fused else 2) * iters
    assert kern.get("fft_cols", (0, 0))[1] == (0 if pc == 2 else iters)
    assert kern.get("fft_rows_fwd", (0, 0))[1] == 0 and kern.get("fft_rows_inv", (0, 0))[1] == 0
    assert kern["shrink_synthesis" if implicit else "synthesis_level"][1] == 2 * iters
    assert ("analysis_level" in kern) == (not implicit)
    # every launch of an iteration is accounted to one phase
    assert sum(v[1] for v in phases.values()) == sum(v[1] for v in kern.values())
    assert abs(sum(v[0] for v in phases.values()) - sum(v[0] for v in kern.values())) < 1e-6


def test_profile_every(mlba):
    """Recording every k-th iteration: the count and the per-launch averages."""
    announce("profile every 3rd iteration")
    n, p = 64, 9
    H = synth.gaussian_psf(p, 1.5)
    g = synth.rng(5).random((n, n))
    with mlba.Plan(n, p, mlba.RECT, mlba.BCCB, 2, cuda(H)) as plan:
        plan.profile_begin(100, every=3)
        plan.restore(cuda(g), alpha=0.05, mu=1e-3, delta=0.3, iters=10, implicit=True)
        _, rec = plan.profile_end()
        kern = plan.profile_kernels()
    assert rec == 4  # iterations 0, 3, 6, 9
    assert kern["conv_blur"][1] == 4 and kern["conv_blur"][0] > 0.0


@pytest.mark.parametrize("bc,pc,method,implicit", [
    ("REFLECT", 0, "MLBA", True),    # BCCB: residual and P row passes fused
    ("REFLECT", 1, "MLBA", False),   # DCT (Algorithm 3): its row passes fused likewise
    ("ZERO", 0, "MLBA", False),
    ("ZERO", 1, "MLBA", True),
    ("PERIODIC", 0, "MLBA", True),   # A = C: the residual formed in the spectrum
    ("PERIODIC", 0, "MLBA", False),
    ("PERIODIC", 1, "MLBA", True),
    ("REFLECT", 1, "ALG4", True),    # Algorithm 4's residual on the grid
    ("ZERO", 0, "ALG4", False),
])
def test_restore_square_models_fft_blur(mlba, bc, pc, method, implicit):
    """MLBA (eq. MLBA2) and Algorithm 4 on the square models with the FFT
    blur, against the oracle; the launches show which path ran."""
    n, p, L, iters = 96, 9, 2, 25
    announce(f"restore {bc} precond={pc} {method} FFT blur implicit={implicit}")
    gen = synth.rng(4600 + n + pc + len(bc))
    H = synth.gaussian_psf(p, 1.5)
    obc = getattr(ob, bc)
    truth = synth.shapes_image(n + p - 1, gen, n_rect=6, n_disk=3)
    g = synth.add_noise(ob.blur(truth, H, ob.RECT), synth.white_noise((n, n), gen), 0.01)
    alphas = np.full(iters, 0.05)
    mu = np.linspace(1e-3, 2e-3, 8 * L + 1)
    alg4 = method == "ALG4"
    with mlba.Plan(n, p, getattr(mlba, bc), pc, L, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        plan.profile_begin(iters)
        if alg4:
            f, info = plan.restore(cuda(g), alpha_table=alphas, mu=mu, delta=1.0, iters=iters, method=mlba.ALG4,
                                   implicit=implicit)
        else:
            deltas = omlba.delta_table(H, n, obc, pc, alphas, 0.0, iters + 1)
            f, info = plan.restore(cuda(g), alpha_table=alphas, mu=mu, delta_table=deltas, iters=iters,
                                   implicit=implicit)
        plan.profile_end()
        kern = plan.profile_kernels()
        f = host(f)
    if alg4:
        ref = oa.alg4(g, H, obc, pc, L, alphas, np.ones(iters + 1), mu, iters)
    else:
        ref = omlba.mlba(g, H, obc, pc, L, alphas, deltas, mu, iters)
    print(f"  image {rel_err(f, ref['f']):.2e} max {max_err(f, ref['f']):.2e} "
          f"rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}; {sorted(kern)}", flush=True)
    assert rel_err(f, ref["f"]) < 1e-4 and max_err(f, ref["f"]) < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4
    spectral = bc == "PERIODIC" and pc == 0
    fused = pc in (0, 1) and not alg4 and not spectral
    assert ("fc_cols" in kern) == (not spectral)
    if spectral:  # one 2-D transform pair per iteration
        assert kern["fft_rows_fwd"][1] == kern["fft_cols"][1] == kern["fft_rows_inv"][1] == iters
    assert kern.get("fc_residual_precond_rows", (0, 0))[1] == (iters if fused else 0)
    assert kern.get("precond_rows_fc_fwd", (0, 0))[1] == (iters if fused else 0)
    if not spectral:
        assert kern["fc_cols"][1] == (1 if alg4 else 2) * iters
