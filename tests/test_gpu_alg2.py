"""Algorithm 2 (section 4.2) on the GPU against the FP64 oracle: the image after
the run within 1e-4, the residual history within 1e-4, and the same number of
PCG steps beta_n at every iteration (cases chosen away from the 1e-3 boundary
are decided identically in FP32 and FP64; the observed ratios are printed)."""
import numpy as np
import pytest

import synth
from oracle import alg2 as oa2
from oracle import blur as ob
from tests._util import announce, cuda, host, max_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("n,p,bc,pc,L,alpha,pcg", [
    (96, 9, ob.RECT, 0, 2, 0.05, (5, 1e-3)),
    (96, 9, ob.RECT, 0, 2, 0.05, (5, 0.05)),     # beta_n varies between 2 and 4
    (128, 17, ob.RECT, 1, 1, 0.02, (5, 1e-3)),
    (96, 9, ob.ZERO, 0, 2, 0.05, (3, 1e-2)),
    (64, 7, ob.REFLECT, 1, 3, 0.1, (5, 1e-3)),
])
def test_alg2_against_oracle(mlba, n, p, bc, pc, L, alpha, pcg, implicit):
    announce(f"Alg2 n={n} p={p} bc={bc} pc={pc} L={L} alpha={alpha} pcg={pcg} implicit={implicit}")
    gen = synth.rng(n + p + bc + 7 * pc)
    truth = synth.shapes_image(n + p - 1, gen, n_rect=6, n_disk=3, n_bumps=3)
    H = synth.motion_psf(p, p - 2.0, gen.uniform(0, np.pi))
    g = synth.add_noise(ob.blur(truth, H, ob.RECT), synth.white_noise((n, n), gen), 0.01)
    iters = 25
    alphas = np.full(iters, alpha)
    deltas = np.full(iters + 1, 0.8)
    mu = 1e-3
    ref = oa2.alg2(g, H, bc, pc, L, alphas, deltas, mu, iters, beta_max=pcg[0], tol=pcg[1])
    with mlba.Plan(n, p, bc, pc, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=mu, delta=0.8, iters=iters, method=mlba.ALG2, pcg=pcg,
                               implicit=implicit)
        f = host(f)
    print(f"  betas gpu {info.pcg_steps} oracle {ref['betas'].tolist()}; image {rel_err(f, ref['f']):.2e}",
          flush=True)
    assert info.pcg_steps == ref["betas"].tolist()
    assert rel_err(f, ref["f"]) < 1e-4 and max_err(f, ref["f"]) < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("n,p,pcg", [(96, 9, (5, 0.05)), (128, 17, (5, 1e-3))])
def test_alg2_with_the_fft_blur(mlba, implicit, n, p, pcg):
    """The PCG's products (A A^T + alpha I) d as one transform pair of the FFT
    grid (|H|^2) with the epilogue + alpha d and d . q, and the final A^T;
    the same beta_n as the oracle and the direct blur."""
    L, alpha = 2, 0.05
    announce(f"Alg2 FFT blur n={n} p={p} pcg={pcg} implicit={implicit}")
    gen = synth.rng(n + p + 11)
    truth = synth.shapes_image(n + p - 1, gen, n_rect=6, n_disk=3, n_bumps=3)
    H = synth.motion_psf(p, p - 2.0, gen.uniform(0, np.pi))
    g = synth.add_noise(ob.blur(truth, H, ob.RECT), synth.white_noise((n, n), gen), 0.01)
    iters = 20
    ref = oa2.alg2(g, H, ob.RECT, 0, L, np.full(iters, alpha), np.full(iters + 1, 0.8), 1e-3, iters,
                   beta_max=pcg[0], tol=pcg[1])
    with mlba.Plan(n, p, ob.RECT, 0, L, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        f, info = plan.restore(cuda(g), alpha=alpha, mu=1e-3, delta=0.8, iters=iters, method=mlba.ALG2, pcg=pcg,
                               implicit=implicit)
        f = host(f)
        plan.set_blur(mlba.BLUR_DIRECT)
        f_d, info_d = plan.restore(cuda(g), alpha=alpha, mu=1e-3, delta=0.8, iters=iters, method=mlba.ALG2,
                                   pcg=pcg, implicit=implicit)
        f_d = host(f_d)
    print(f"  betas gpu {info.pcg_steps} oracle {ref['betas'].tolist()}; image {rel_err(f, ref['f']):.2e} "
          f"max {max_err(f, ref['f']):.2e}; vs direct {rel_err(f, f_d):.2e}", flush=True)
    assert info.pcg_steps == ref["betas"].tolist() == info_d.pcg_steps
    assert rel_err(f, ref["f"]) < 1e-4 and max_err(f, ref["f"]) < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4
    assert rel_err(f, f_d) < 1e-4


def test_alg2_exact_preconditioner_takes_one_step(mlba):
    """Periodic model, BCCB plan: the preconditioner is exact, every beta_n = 1,
    and the run equals the plain preconditioned MLBA."""
    announce("Alg2 with an exact preconditioner")
    n, p, L, iters = 64, 7, 2, 15
    gen = synth.rng(2)
    H = synth.gaussian_psf(p, 1.5)
    g = synth.rng(3).standard_normal((n, n))
    with mlba.Plan(n, p, ob.PERIODIC, 0, L, cuda(H)) as plan:
        f2, i2 = plan.restore(cuda(g), alpha=0.05, mu=1e-3, delta=0.5, iters=iters, method=mlba.ALG2)
        f1, i1 = plan.restore(cuda(g), alpha=0.05, mu=1e-3, delta=0.5, iters=iters)
        f1, f2 = host(f1), host(f2)
    assert i2.pcg_steps == [1] * iters
    assert rel_err(f2, f1) < 1e-5


def test_alg2_needs_a_spectral_preconditioner(mlba):
    from paper_1504_07234_amd import _lib
    announce("Alg2 argument checks")
    with mlba.Plan(32, 5, ob.RECT, 2, 1, cuda(synth.gaussian_psf(5, 1.0))) as plan:
        with pytest.raises(_lib.MLBAError) as e:
            plan.restore(cuda(np.zeros((32, 32))), alpha=0.1, iters=2, method=mlba.ALG2)
        assert e.value.status == _lib.EUNSUPPORTED
