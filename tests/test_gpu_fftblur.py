"""The rectangular model's blur A and its transpose computed by FFTs of an
M x M grid (section 2.1), against the FP64 oracle; and the restoration with
it.  Bars: 1e-5 (relative, L2) per operator, 1e-4 on restored images."""
import numpy as np
import pytest

import synth
from oracle import blur as ob
from oracle import mlba as omlba
from tests._util import announce, cuda, host, max_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


# (n, p): ragged grids, odd N, the largest PSF, the 3072-point limit, the bench shape
CASES = [(8, 1), (64, 9), (100, 17), (97, 5), (256, 49), (2048, 31), (3000, 49)]


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


def test_fft_blur_needs_rect_and_fits(mlba):
    from paper_1504_07234_amd import _lib
    announce("FFT blur argument checks")
    H = cuda(synth.gaussian_psf(5, 1.0))
    with mlba.Plan(64, 5, mlba.REFLECT, mlba.NONE, 1, H) as plan:
        with pytest.raises(_lib.MLBAError) as e:
            plan.set_blur(mlba.BLUR_FFT)
        assert e.value.status == _lib.EUNSUPPORTED
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
    assert rel_err(f, ref["f"]) < 1e-4
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
