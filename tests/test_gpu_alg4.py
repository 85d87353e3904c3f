"""Algorithm 4 and 4-NS (section 5) on the GPU against the FP64 oracle.

Bars: the direction C^T (C C^T + alpha I)^{-1} r within 1e-5 (relative, L2);
restored images within 1e-4 of the oracle after the full run, both states;
4-NS: the same stopping index; every alpha_n within 1e-5 + 1e-6 kappa_n
relative, kappa_n = |d log alpha_n / d log q_n| (the equation for alpha_n
becomes ill-conditioned as q_n -> 1 near the stop, where an FP32 residual norm
moves it by ~1e-7 kappa_n); the image within 1e-4.
"""
import numpy as np
import pytest

import synth
from oracle import alg4 as oa
from oracle import blur as ob
from tests._util import announce, cuda, host, max_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


def _problem(n, p, bc, sym, seed):
    g = synth.rng(seed)
    truth = synth.shapes_image(n, g, n_rect=8, n_disk=4, n_bumps=3)
    H = synth.gaussian_psf(p, 2.0) if sym else synth.motion_psf(p, p - 2.0, g.uniform(0, np.pi))
    b = ob.blur(truth, H, bc)
    return synth.add_noise(b, synth.white_noise((n, n), g), 0.01), H, synth.noise_norm(b, 0.01), truth


@pytest.mark.parametrize("n", [8, 14, 64, 96, 192, 196, 256, 512])  # 14, 196: Bluestein-form transforms
@pytest.mark.parametrize("kind,bc", [(oa.BCCB, ob.ZERO), (oa.BCCB, ob.PERIODIC), (oa.DCT, ob.REFLECT)])
def test_direction_operator(mlba, n, kind, bc):
    p = min(9, n - 1 if (n - 1) % 2 else n - 2)
    announce(f"C^T (CC^T + alpha)^-1 n={n} kind={kind} bc={bc}")
    H = synth.motion_psf(p, p - 2.0, 0.7)  # nonsymmetric: the phase of Lambda_c matters
    r = synth.rng(n).standard_normal((n, n))
    with mlba.Plan(n, p, bc, kind, 1, cuda(H)) as plan:
        t = host(plan.apply_CtP(cuda(r), 0.03))
    ref = oa.apply_ct_prec(r, H, 0.03, kind)
    assert rel_err(t, ref) < 1e-5 and max_err(t, ref) < 1e-4


def test_direction_rejects_rect(mlba):
    from paper_1504_07234_amd import _lib
    announce("C^T P on a rectangular plan")
    with mlba.Plan(32, 5, mlba.RECT, mlba.BCCB, 1, cuda(synth.gaussian_psf(5, 1.0))) as plan:
        with pytest.raises(_lib.MLBAError) as e:
            plan.apply_CtP(cuda(np.zeros((32, 32))), 0.1)
        assert e.value.status == _lib.EUNSUPPORTED


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("bc,kind,sym,alpha,iters,L,n", [
    (ob.PERIODIC, oa.BCCB, False, 0.01, 100, 2, 128),
    (ob.ZERO, oa.BCCB, False, 0.05, 40, 2, 96),
    (ob.REFLECT, oa.DCT, True, 0.05, 100, 3, 128),
    (ob.REFLECT, oa.BCCB, False, 0.05, 60, 1, 64),
])
def test_alg4_against_oracle(mlba, bc, kind, sym, alpha, iters, L, n, implicit):
    p = 9
    announce(f"Alg4 bc={bc} kind={kind} alpha={alpha} iters={iters} L={L} n={n} implicit={implicit}")
    g, H, _, _ = _problem(n, p, bc, sym, 40 + bc + kind)
    mu = np.linspace(1e-3, 2e-3, 8 * L + 1)
    ref = oa.alg4(g, H, bc, kind, L, np.full(iters, alpha), np.ones(iters + 1), mu, iters)
    with mlba.Plan(n, p, bc, kind, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=mu, delta=1.0, iters=iters, method=mlba.ALG4,
                               implicit=implicit)
        f = host(f)
    e = rel_err(f, ref["f"])
    print(f"  image rel err {e:.2e} rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4
    assert np.allclose(info.alphas, alpha)


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("n,p,L,iters", [(2048, 31, 3, 4), (250, 17, 2, 60), (96, 5, 1, 80)])
def test_alg4_periodic_spectral_residual(mlba, n, p, L, iters, implicit):
    """Periodic model with the BCCB matrix: A = C, the residual formed in the
    spectrum (F g - Lambda_c F u, ||r|| by Parseval) and one transform pair per
    iteration; the 2048 case is the bench's Algorithm 4 shape (31 x 31 disk,
    3 levels), 250 a 2/5-smooth run-time length.  Image and residual norms
    against the oracle, which forms r = g - C u with the periodic blur."""
    announce(f"Alg4 periodic spectral residual n={n} p={p} L={L} iters={iters} implicit={implicit}")
    gen = synth.rng(900 + n)
    truth = synth.shapes_image(n, gen, n_rect=8, n_disk=4, n_bumps=3)
    H = synth.disk_psf(p, (p - 1) / 2.0) if p > 9 else synth.motion_psf(p, p - 2.0, 0.4)
    b = ob.blur(truth, H, ob.PERIODIC)
    g = synth.add_noise(b, synth.white_noise((n, n), gen), 0.01)
    alpha, mu = 0.02, np.linspace(1e-3, 2e-3, 8 * L + 1)
    ref = oa.alg4(g, H, ob.PERIODIC, oa.BCCB, L, np.full(iters, alpha), np.ones(iters + 1), mu, iters)
    with mlba.Plan(n, p, ob.PERIODIC, oa.BCCB, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=mu, delta=1.0, iters=iters, method=mlba.ALG4,
                               implicit=implicit)
        f = host(f)
    e, em, er = rel_err(f, ref["f"]), max_err(f, ref["f"]), rel_err(info.rnorm, ref["rnorm"])
    print(f"  image rel {e:.2e} max {em:.2e} rnorm {er:.2e}", flush=True)
    assert e < 1e-4 and em < 1e-4
    assert er < 1e-4


def _alpha_condition(g, H, bc, L, mu, alphas, kind=None):
    """kappa_n = |d log alpha_n / d log q_n| along the oracle's 4-NS run.

    alpha_n solves alpha^2 S0(alpha) = q_n^2 R (S0 = sum w / (s + alpha)^2), so
    d log alpha / d log q = 2 / (2 S1 / S0), S1 = sum w s / (s + alpha)^3.  Near
    the stop q_n -> 1 and kappa_n grows by orders of magnitude: a relative
    change of q_n (through ||r^n||) of 1e-7 then moves alpha_n by ~1e-7 kappa_n."""
    from oracle import framelet as ofr
    from oracle.mlba import soft_threshold
    import scipy.fft
    from oracle import precond as opc
    kind = oa.BCCB if kind is None else kind
    n = g.shape[0]
    if kind == oa.BCCB:
        s = np.abs(oa.centred_eigs(H, n)) ** 2
    else:
        s = opc.dct_eigs(opc.symmetrize(H), n) ** 2
    z = np.zeros((8 * L + 1, n, n))
    out = []
    for a in alphas:
        r = g - ob.blur(ofr.synthesis(soft_threshold(z, mu), L), H, bc)
        w = np.abs(np.fft.fft2(r)) ** 2 if kind == oa.BCCB else scipy.fft.dctn(r, type=2, norm="ortho") ** 2
        S0 = np.sum(w / (s + a) ** 2)
        S1 = np.sum(w * s / (s + a) ** 3)
        out.append(S0 / S1)
        z = z + ofr.analysis(oa.apply_ct_prec(r, H, a, kind), L)
    return np.asarray(out)


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("bc,n,L,kind", [(ob.ZERO, 128, 2, oa.BCCB), (ob.PERIODIC, 96, 1, oa.BCCB),
                                         (ob.REFLECT, 192, 2, oa.BCCB), (ob.REFLECT, 128, 2, oa.DCT),
                                         (ob.ANTIREFLECT, 96, 2, oa.DCT),
                                         # 196: Bluestein-form transforms (stops 1e-3 and 5e-4 clear of the bound)
                                         (ob.PERIODIC, 196, 1, oa.BCCB), (ob.REFLECT, 196, 2, oa.DCT)])
def test_alg4_ns_against_oracle(mlba, bc, n, L, kind, implicit):
    """4-NS with the BCCB spectrum and with the DCT of the symmetrised PSF
    (Alg-BC4-NS of Example 4: antireflective model, Gaussian PSF, DCT)."""
    p = 9
    announce(f"Alg4-NS bc={bc} n={n} L={L} kind={kind} implicit={implicit}")
    g, H, noise, _ = _problem(n, p, bc, kind == oa.DCT, 70 + bc)
    mu = 1e-3
    ref = oa.alg4_ns(g, H, bc, kind, L, mu, noise, q=0.5, rho=1e-4, max_iters=300)
    k = ref["iters"]
    assert 0 < k < 300
    with mlba.Plan(n, p, bc, kind, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=0.5, mu=mu, delta=1.0, iters=300, method=mlba.ALG4,
                               implicit=implicit, ns=(0.5, 1e-4), stop=(noise, 0.0, 1))
        f = host(f)
    print(f"  stop gpu {info.iters_done} oracle {k}; alpha rel {rel_err(info.alphas, ref['alphas']):.2e}; "
          f"image {rel_err(f, ref['f']):.2e}", flush=True)
    assert info.iters_done == k
    # alpha_n within FP32 round-off carried through the condition of its equation
    kappa = _alpha_condition(g, H, bc, L, mu, ref["alphas"], kind)
    dev = np.abs(np.asarray(info.alphas) - ref["alphas"]) / ref["alphas"]
    print(f"  alpha rel dev {np.array2string(dev, precision=1)} kappa {np.array2string(kappa, precision=1)}",
          flush=True)
    assert np.all(dev <= 1e-5 + 1e-6 * kappa)
    assert rel_err(f, ref["f"]) < 1e-4 and max_err(f, ref["f"]) < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"][:k]) < 1e-4


@pytest.mark.parametrize("kind", [oa.BCCB, oa.DCT])
def test_alg4_ns_first_steps_at_2048(mlba, kind):
    """The 2048 observation (the compiled 2048-point transforms, including the
    DCT's split column pass): the first three 4-NS steps, far from the stop
    where alpha_n is well conditioned, against the oracle."""
    n, p, L, iters = 2048, 9, 2, 3
    bc = ob.REFLECT
    announce(f"Alg4-NS first steps n={n} kind={kind}")
    g, H, noise, _ = _problem(n, p, bc, True, 91 + kind)
    ref = oa.alg4_ns(g, H, bc, kind, L, 1e-3, noise, q=0.5, rho=1e-4, max_iters=iters)
    assert ref["iters"] == iters  # the stop does not fire this early
    with mlba.Plan(n, p, bc, kind, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=0.5, mu=1e-3, delta=1.0, iters=iters, method=mlba.ALG4,
                               implicit=True, ns=(0.5, 1e-4), stop=(noise, 0.0, 1))
        f = host(f)
    print(f"  alphas gpu {info.alphas} oracle {ref['alphas'].tolist()}; image {rel_err(f, ref['f']):.2e}",
          flush=True)
    assert info.iters_done == iters
    assert rel_err(info.alphas, ref["alphas"]) < 1e-4
    assert rel_err(f, ref["f"]) < 1e-4 and max_err(f, ref["f"]) < 1e-4


def test_alg4_rejections(mlba):
    from paper_1504_07234_amd import _lib
    announce("Alg4 argument checks")
    H = cuda(synth.gaussian_psf(5, 1.0))
    g = cuda(np.zeros((32, 32)))
    with mlba.Plan(32, 5, mlba.RECT, mlba.BCCB, 1, H) as plan:
        with pytest.raises(_lib.MLBAError) as e:
            plan.restore(g, alpha=0.1, iters=2, method=mlba.ALG4)
        assert e.value.status == _lib.EUNSUPPORTED
    with mlba.Plan(33, 5, mlba.ANTIREFLECT, mlba.AR, 1, H) as plan:
        with pytest.raises(_lib.MLBAError) as e:  # 4-NS needs an orthogonal transform (Parseval)
            plan.restore(cuda(np.zeros((33, 33))), alpha=0.1, iters=2, method=mlba.ALG4, ns=(0.5, 1e-4),
                         stop=(1.0, 0.0, 1))
        assert e.value.status == _lib.EUNSUPPORTED
    with mlba.Plan(32, 5, mlba.ZERO, mlba.BCCB, 1, H) as plan:
        with pytest.raises(_lib.MLBAError) as e:  # no noise level
            plan.restore(g, alpha=0.1, iters=2, method=mlba.ALG4, ns=(0.5, 1e-4))
        assert e.value.status == _lib.EINVAL
        with pytest.raises(_lib.MLBAError):  # q must exceed 2 rho
            plan.restore(g, alpha=0.1, iters=2, method=mlba.ALG4, ns=(1e-4, 1e-3), stop=(1.0, 0.0, 1))
