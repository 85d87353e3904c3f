"""Antireflective boundary conditions (sections 2.2, 4.3) on the GPU against
the FP64 oracle: the blur A under the antireflective pad, the reblurring A'
that replaces A^T, the antireflective-transform preconditioner
(Q Q' + alpha I)^-1 and the Algorithm 4 direction Q'(Q Q' + alpha I)^-1, and
whole runs of eq. (MLBA2), Algorithm 4 and Algorithm 2 with this model.

Bars: operators 1e-5 relative L2 and 1e-4 max relative to the oracle's
largest entry; restored images 1e-4 relative L2."""
import numpy as np
import pytest

import synth
from oracle import alg2 as oa2
from oracle import alg4 as oa4
from oracle import blur as ob
from oracle import mlba as omlba
from oracle import precond as opc
from tests._util import announce, cuda, host, max_err, rel_err

pytestmark = pytest.mark.gpu

AR_BC = ob.ANTIREFLECT
TOL_L2 = 1e-5
TOL_MAX = 1e-4


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


def _psf(kind, p, seed):
    g = synth.rng(seed)
    if kind == "gauss":
        return synth.gaussian_psf(p, p / 5.0 + 0.5)
    if kind == "motion":
        return synth.motion_psf(p, p - 2.0, g.uniform(0, np.pi))
    h = g.random((p, p))
    return h / h.sum()


@pytest.mark.parametrize("n,p,kind", [
    (64, 9, "gauss"),
    (100, 7, "rand"),
    (96, 17, "motion"),
    (150, 31, "motion"),   # several tiles and a ragged tail
    (77, 35, "rand"),      # the generic tap loop
    (100, 49, "rand"),     # the largest PSF (pad of 24)
    (33, 1, "rand"),
    (9, 9, "rand"),        # the pad as wide as the image allows (c = n - 1 - 4)
    (5, 3, "rand"),
])
def test_blur_and_reblur(mlba, n, p, kind):
    announce(f"antireflective blur/reblur n={n} p={p} {kind}")
    H = _psf(kind, p, n + 3 * p)
    g = synth.rng(4000 + n + p)
    u = g.random((n, n))
    y = g.standard_normal((n, n))
    gi = g.random((n, n))
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.NONE, 1, cuda(H)) as plan:
        Au = host(plan.apply_A(cuda(u)))
        Ary = host(plan.apply_At(cuda(y)))
        r = host(plan.residual(cuda(gi), cuda(u)))
    ref_Au = ob.blur(u, H, AR_BC)
    ref_Ary = ob.reblur(y, H, AR_BC)
    print(f"  A {rel_err(Au, ref_Au):.2e}  A' {rel_err(Ary, ref_Ary):.2e}", flush=True)
    assert rel_err(Au, ref_Au) < TOL_L2 and max_err(Au, ref_Au) < TOL_MAX
    assert rel_err(Ary, ref_Ary) < TOL_L2 and max_err(Ary, ref_Ary) < TOL_MAX
    assert rel_err(r, gi - ref_Au) < TOL_L2


@pytest.mark.parametrize("n,p,kind", [
    (64, 9, "gauss"),
    (97, 31, "motion"),
    (150, 17, "rand"),
    (257, 41, "rand"),
    (200, 49, "rand"),     # the largest PSF
    (1025, 31, "gauss"),   # the antireflective workload's shapes (grid 1152)
])
def test_fft_grid_blur_and_reblur(mlba, n, p, kind):
    """A and A' with the antireflective extension placed on the FFT grid."""
    announce(f"antireflective FFT-grid blur/reblur n={n} p={p} {kind}")
    H = _psf(kind, p, n + 5 * p)
    g = synth.rng(4500 + n + p)
    u = g.random((n, n))
    y = g.standard_normal((n, n))
    gi = g.random((n, n))
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.NONE, 1, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        Au = host(plan.apply_A(cuda(u)))
        Ary = host(plan.apply_At(cuda(y)))
        r = host(plan.residual(cuda(gi), cuda(u)))
    ref_Au = ob.blur(u, H, AR_BC)
    ref_Ary = ob.reblur(y, H, AR_BC)
    print(f"  A {rel_err(Au, ref_Au):.2e}  A' {rel_err(Ary, ref_Ary):.2e}", flush=True)
    assert rel_err(Au, ref_Au) < TOL_L2 and max_err(Au, ref_Au) < TOL_MAX
    assert rel_err(Ary, ref_Ary) < TOL_L2 and max_err(Ary, ref_Ary) < TOL_MAX
    assert rel_err(r, gi - ref_Au) < TOL_L2


def test_affine_image_is_blurred_exactly(mlba):
    """An affine image under a normalised symmetric PSF is left unchanged by
    the antireflective blur, borders included (the pad continues it)."""
    n, p = 130, 15
    announce("antireflective blur of an affine image")
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    f = 0.2 + 0.003 * yy - 0.002 * xx
    H = synth.gaussian_psf(p, 2.5)
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.NONE, 1, cuda(H)) as plan:
        Af = host(plan.apply_A(cuda(f)))
    assert np.abs(Af - f).max() < 2e-6


# transform lengths 2^a 3^b 5^c, and (8, 15, 196, 500: lengths 14, 28, 390, 998)
# the Bluestein form over m = 27, 60, 800, 2000
AR_SIZES = [4, 6, 8, 10, 11, 13, 15, 51, 65, 97, 193, 196, 226, 257, 433, 500, 1025]


@pytest.mark.parametrize("n", AR_SIZES)
def test_ar_preconditioner(mlba, n):
    p = min(9, n - 1 if (n - 1) % 2 else n - 2)
    announce(f"antireflective preconditioner n={n} p={p}")
    H = _psf("motion" if p >= 5 else "rand", p, n)  # nonsymmetric: symmetrised inside
    g = synth.rng(5000 + n)
    smooth = synth.shapes_image(n, g, n_rect=6, n_disk=3, n_bumps=3)
    noise = g.standard_normal((n, n))
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, 1, cuda(H)) as plan:
        for alpha in (0.5, 0.02):
            for r in (smooth, noise):
                got = host(plan.apply_P(cuda(r), alpha))
                ref = opc.apply(r, H, alpha, opc.AR)
                e2, em = rel_err(got, ref), max_err(got, ref)
                print(f"  alpha={alpha} l2={e2:.2e} max={em:.2e}", flush=True)
                assert e2 < TOL_L2 and em < TOL_MAX


def test_set_psf_recomputes_the_antireflective_spectra(mlba):
    """A new PSF replaces the transform's eigenvalues and the FFT grid's
    spectrum: P, A and A' follow it."""
    n, p = 97, 9
    announce("antireflective set_psf")
    H1 = _psf("gauss", p, 1)
    H2 = _psf("motion", p, 2)
    g = synth.rng(7)
    r = g.standard_normal((n, n))
    u = g.random((n, n))
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, 1, cuda(H1)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        plan.apply_P(cuda(r), 0.05)
        plan.set_psf(cuda(H2))
        t = host(plan.apply_P(cuda(r), 0.05))
        Au = host(plan.apply_A(cuda(u)))
        Ary = host(plan.apply_At(cuda(r)))
    assert rel_err(t, opc.apply_ar(r, H2, 0.05)) < TOL_L2
    assert rel_err(Au, ob.blur(u, H2, AR_BC)) < TOL_L2
    assert rel_err(Ary, ob.reblur(r, H2, AR_BC)) < TOL_L2


def test_ar_preconditioner_in_place(mlba):
    n, p = 97, 7
    announce("antireflective preconditioner in place")
    H = _psf("rand", p, 6)
    r = synth.rng(6).standard_normal((n, n))
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, 1, cuda(H)) as plan:
        t = cuda(r)
        plan.apply_P(t, 0.1, out=t)
        assert rel_err(host(t), opc.apply_ar(r, H, 0.1)) < TOL_L2


@pytest.mark.parametrize("n", [13, 97, 257])
def test_ar_direction(mlba, n):
    p = 9
    announce(f"antireflective Q'(QQ' + alpha)^-1 n={n}")
    H = synth.motion_psf(p, p - 2.0, 0.7)
    r = synth.rng(n + 1).standard_normal((n, n))
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, 1, cuda(H)) as plan:
        t = host(plan.apply_CtP(cuda(r), 0.03))
    ref = oa4.apply_ct_prec(r, H, 0.03, oa4.AR)
    assert rel_err(t, ref) < TOL_L2 and max_err(t, ref) < TOL_MAX


@pytest.mark.parametrize("n", [600, 2049, 3])
def test_ar_sizes_outside_the_transform(mlba, n):
    """The transform length 2(n - 1) must fit one workgroup: at most 2048 when
    it is 2^a 3^b 5^c, else its Bluestein length (600: 1198 = 2 * 599 needs
    2400); n >= 4."""
    from paper_1504_07234_amd import _lib
    announce(f"antireflective transform size n={n}")
    with pytest.raises(_lib.MLBAError) as e:
        mlba.Plan(n, 3, mlba.ANTIREFLECT, mlba.AR, 1, cuda(synth.gaussian_psf(3, 1.0)))
    assert e.value.status == _lib.EUNSUPPORTED


def _sym_opnorm(H, n, alpha):
    """||A' P A|| for a quadrantally symmetric PSF and the antireflective
    preconditioner: A = A' = Q = T Lambda T^-1, so the operator is
    T Lambda^2 (Lambda^2 + alpha)^-1 T^-1 (pinned against Arnoldi on the CPU)."""
    lam = opc.ar_eigs(H, n)
    return float((lam * lam / (lam * lam + alpha)).max())


def test_opnorm_of_the_reblurred_operator(mlba):
    """A' P A is not normal (T is not orthogonal): the power iteration's
    ||M v|| / ||v|| approaches the spectral radius but may exceed it while the
    slow components (eigenvalues clustered at the top) have not died out.  An
    overestimate only shortens the automatic step, so the bar allows 1 % above
    and 3 % below."""
    n, p = 65, 9
    announce("||A' P A|| antireflective")
    H = synth.gaussian_psf(p, 2.0)
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, 1, cuda(H)) as plan:
        got = plan.opnorm(0.05, 200)
    ref = _sym_opnorm(H, n, 0.05)
    print(f"  gpu={got:.6f} oracle={ref:.6f}", flush=True)
    assert ref * 0.97 <= got <= ref * 1.01


def _problem(n, p, sym, seed, level=0.01):
    """The observation is the valid part of a larger scene (section 6's
    examples): truth (n + p - 1)^2, blurred with the rectangular model."""
    g = synth.rng(seed)
    truth = synth.shapes_image(n + p - 1, g, n_rect=8, n_disk=4, n_bumps=3)
    H = synth.gaussian_psf(p, 2.5) if sym else synth.motion_psf(p, p - 2.0, g.uniform(0, np.pi))
    b = ob.blur(truth, H, ob.RECT)
    return synth.add_noise(b, synth.white_noise((n, n), g), level), H


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("n,p,pc,sym,L,alpha,iters", [
    (97, 9, opc.AR, False, 2, 0.02, 40),    # Alg-BC3
    (96, 9, opc.BCCB, False, 2, 0.37, 40),  # Alg-BC1 (Example 3's alpha)
    (96, 11, opc.DCT, True, 1, 0.05, 30),   # Alg-BC1 with the DCT (Example 4)
    (80, 7, opc.NONE, False, 3, 0.0, 30),
    (65, 13, opc.AR, True, 3, 0.01, 25),
])
def test_mlba_antireflective_against_oracle(mlba, n, p, pc, sym, L, alpha, iters, implicit):
    """The automatic step 0.9 / max(||A' P A||, 0.9) from the oracle's norm:
    with a periodic or reflective preconditioner the antireflective model's
    norm reaches several units (6 to 15 here) and a fixed step diverges."""
    announce(f"MLBA antireflective n={n} p={p} pc={pc} L={L} implicit={implicit}")
    g, H = _problem(n, p, sym, 60 + n + pc)
    mu = 1e-3
    delta = omlba.delta_auto(omlba.opnorm(H, n, AR_BC, pc, alpha, tol=1e-6))
    ref = omlba.mlba(g, H, AR_BC, pc, L, np.full(iters, alpha), np.full(iters + 1, delta), mu, iters)
    with mlba.Plan(n, p, mlba.ANTIREFLECT, pc, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=mu, delta=delta, iters=iters, implicit=implicit)
        f = host(f)
    e = rel_err(f, ref["f"])
    print(f"  image {e:.2e} rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


@pytest.mark.parametrize("blur", ["direct", "fft"])
def test_example4_shape(mlba, blur):
    """Example 4's shape: a 226 x 226 observation of a larger scene, 31 x 31
    Gaussian of standard deviation 2.5, 2 % noise, antireflective conditions
    with the antireflective-transform preconditioner (transform length 450 =
    2 * 3^2 * 5^2), alpha = 0.01 (Table 4's Alg-BC3), automatic step."""
    n, p, L, iters, alpha = 226, 31, 2, 20, 0.01
    announce(f"Example 4 shape n={n} p={p} blur={blur}")
    g0 = synth.rng(226)
    truth = synth.shapes_image(n + p - 1, g0, n_rect=8, n_disk=4, n_bumps=3)
    H = synth.gaussian_psf(p, 2.5)
    g = synth.add_noise(ob.blur(truth, H, ob.RECT), synth.white_noise((n, n), g0), 0.02)
    delta = omlba.delta_auto(_sym_opnorm(H, n, alpha))
    ref = omlba.mlba(g, H, AR_BC, opc.AR, L, np.full(iters, alpha), np.full(iters + 1, delta), 1e-3, iters)
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, L, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT if blur == "fft" else mlba.BLUR_DIRECT)
        f, info = plan.restore(cuda(g), alpha=alpha, mu=1e-3, delta=delta, iters=iters, implicit=True)
        f = host(f)
    e = rel_err(f, ref["f"])
    print(f"  image {e:.2e} rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("pc", [opc.AR, opc.BCCB])
def test_mlba_antireflective_fft_blur(mlba, pc, implicit):
    """Whole runs with A and A' on the FFT grid against the oracle; with the
    antireflective transform the residual's inverse row pass runs with the
    transform's forward row pass (kernel counts of the profiled run)."""
    n, p, L, iters = (97, 31, 2, 30) if pc == opc.AR else (96, 25, 2, 30)
    alpha = 0.02 if pc == opc.AR else 0.37
    announce(f"MLBA antireflective FFT blur n={n} p={p} pc={pc} implicit={implicit}")
    g, H = _problem(n, p, pc == opc.AR, 90 + n)
    delta = omlba.delta_auto(omlba.opnorm(H, n, AR_BC, pc, alpha, tol=1e-6))
    ref = omlba.mlba(g, H, AR_BC, pc, L, np.full(iters, alpha), np.full(iters + 1, delta), 1e-3, iters)
    with mlba.Plan(n, p, mlba.ANTIREFLECT, pc, L, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        plan.profile_begin(iters)
        f, info = plan.restore(cuda(g), alpha=alpha, mu=1e-3, delta=delta, iters=iters, implicit=implicit)
        plan.profile_end()
        kern = plan.profile_kernels()
        f = host(f)
    fused = pc == opc.AR
    assert kern.get("fc_residual_precond_rows", (0, 0))[1] == (iters if fused else 0)
    assert kern.get("fc_rows_inv", (0, 0))[1] == (1 if fused else 2) * iters
    assert kern.get("reduce", (0, 0))[1] == (0 if fused else iters)
    e = rel_err(f, ref["f"])
    print(f"  image {e:.2e} rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("n,p,pc,sym", [(97, 9, opc.AR, True), (96, 9, opc.DCT, True)])
def test_alg4_antireflective_against_oracle(mlba, n, p, pc, sym, implicit):
    """Alg-BC4 of Example 4 (Gaussian PSF), with the antireflective transform
    and with the DCT."""
    iters, L, alpha = 40, 2, 0.03
    announce(f"Alg4 antireflective n={n} pc={pc} implicit={implicit}")
    g, H = _problem(n, p, sym, 70 + n + pc)
    mu = np.linspace(1e-3, 2e-3, 8 * L + 1)
    ref = oa4.alg4(g, H, AR_BC, pc, L, np.full(iters, alpha), np.ones(iters + 1), mu, iters)
    with mlba.Plan(n, p, mlba.ANTIREFLECT, pc, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=mu, delta=1.0, iters=iters, method=mlba.ALG4,
                               implicit=implicit)
        f = host(f)
    e = rel_err(f, ref["f"])
    print(f"  image {e:.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


@pytest.mark.parametrize("implicit", [False, True])
def test_alg4_antireflective_fft_grid(mlba, implicit):
    """Alg-BC4 with A on the FFT grid: the residual's inverse row pass fused
    with the transform's forward row pass, the direction
    Q'(Q Q' + alpha I)^{-1} r added straight into the state."""
    n, p, L, alpha, iters = 97, 25, 2, 0.03, 30
    announce(f"Alg4 antireflective FFT grid implicit={implicit}")
    g, H = _problem(n, p, True, 95)
    mu = np.linspace(1e-3, 2e-3, 8 * L + 1)
    ref = oa4.alg4(g, H, AR_BC, opc.AR, L, np.full(iters, alpha), np.ones(iters + 1), mu, iters)
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, L, cuda(H)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        plan.profile_begin(iters)
        f, info = plan.restore(cuda(g), alpha=alpha, mu=mu, delta=1.0, iters=iters, method=mlba.ALG4,
                               implicit=implicit)
        plan.profile_end()
        kern = plan.profile_kernels()
        f = host(f)
    assert kern["fc_residual_precond_rows"][1] == iters and "reduce" not in kern
    assert kern.get("fc_rows_inv", (0, 0))[1] == 0  # no A' product
    e = rel_err(f, ref["f"])
    print(f"  image {e:.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


def test_alg2_antireflective_against_oracle(mlba):
    """Alg-BC2 of Example 3: CG on A A' + alpha I preconditioned by the BCCB
    matrix, A' the reblur (the paper runs it although A A' is not symmetric);
    a Gaussian PSF, where the steps beta_n vary between 3 and 5."""
    n, p, L, alpha, pcg, iters, delta = 96, 9, 2, 0.2, (5, 0.05), 15, 0.5
    announce("Alg2 antireflective")
    g, H = _problem(n, p, True, 81)
    ref = oa2.alg2(g, H, AR_BC, opc.BCCB, L, np.full(iters, alpha), np.full(iters + 1, delta), 1e-3, iters,
                   beta_max=pcg[0], tol=pcg[1])
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.BCCB, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=1e-3, delta=delta, iters=iters, method=mlba.ALG2,
                               pcg=pcg)
        f = host(f)
    print(f"  betas gpu {info.pcg_steps} oracle {ref['betas'].tolist()}; image {rel_err(f, ref['f']):.2e}",
          flush=True)
    assert info.pcg_steps == ref["betas"].tolist()
    assert rel_err(f, ref["f"]) < 1e-4 and max_err(f, ref["f"]) < 1e-4


def test_alg2_with_the_exact_antireflective_preconditioner(mlba):
    """Example 4's remark: with a symmetric PSF the antireflective transform
    preconditioner is (A A' + alpha I)^{-1} itself, so Algorithm 2 takes one
    PCG step per iteration and equals Alg-BC3 (the MLBA with that
    preconditioner); both against the oracle."""
    n, p, L, alpha, delta, iters = 97, 9, 2, 0.05, 0.5, 15
    announce("Alg2 with the exact antireflective preconditioner")
    g, H = _problem(n, p, True, 83)
    ref = oa2.alg2(g, H, AR_BC, opc.AR, L, np.full(iters, alpha), np.full(iters + 1, delta), 1e-3, iters,
                   beta_max=5, tol=0.05)
    assert ref["betas"].tolist() == [1] * iters
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, L, cuda(H)) as plan:
        f2, i2 = plan.restore(cuda(g), alpha=alpha, mu=1e-3, delta=delta, iters=iters, method=mlba.ALG2,
                              pcg=(5, 0.05))
        f1, _ = plan.restore(cuda(g), alpha=alpha, mu=1e-3, delta=delta, iters=iters)
        f1, f2 = host(f1), host(f2)
    assert i2.pcg_steps == [1] * iters
    assert rel_err(f2, ref["f"]) < 1e-4
    assert rel_err(f2, f1) < 1e-5


def test_full_size_antireflective(mlba):
    """The antireflective workload at its full size (n = 1025, 31 x 31
    Gaussian, 3 levels, automatic step) for a few iterations, the image and
    residual history against the oracle."""
    w = synth.make_workload("antireflect-ar-1025")
    iters = 6
    announce(f"antireflective full size n={w.n} p={w.p} L={w.levels} iters={iters}")
    g = synth.add_noise(ob.blur(w.truth, w.psf, ob.RECT), w.xi, w.noise_level)
    d = omlba.delta_auto(_sym_opnorm(w.psf, w.n, w.alpha0))
    ref = omlba.mlba(g, w.psf, AR_BC, opc.AR, w.levels, np.full(iters, w.alpha0), np.full(iters + 1, d), w.mu,
                     iters)
    with mlba.Plan(w.n, w.p, mlba.ANTIREFLECT, mlba.AR, w.levels, cuda(w.psf)) as plan:
        choice = plan.autotune(reps=3)["blur"]  # the blur the timed section runs
        f, info = plan.restore(cuda(g), alpha=w.alpha0, mu=w.mu, delta=d, iters=iters, implicit=True)
        f = host(f)
    print(f"  blur {choice}", flush=True)
    e = rel_err(f, ref["f"])
    print(f"  delta {d:.6f} image {e:.2e} rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


def test_batched_ar_preconditioner(mlba):
    """A batch of antireflective images with the antireflective-transform
    preconditioner (sizes 65 .. 226, one graph replay): equal to the per-image
    path bit for bit, and one image against the oracle."""
    import torch
    announce("batched antireflective transform preconditioner")
    specs = [(65, 9), (97, 7), (129, 15), (226, 11)]
    plans, gs, Hs = [], [], []
    for i, (n, p) in enumerate(specs):
        g, H = _problem(n, p, i % 2 == 0, 300 + i)
        plans.append(mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.AR, 2, cuda(H)))
        gs.append(g)
        Hs.append(H)
    iters, alpha, delta = 12, 0.05, 0.5
    gdev = [cuda(g) for g in gs]
    ref = [pl.restore(g, alpha=alpha, mu=1e-3, delta=delta, iters=iters)[0].clone() for pl, g in zip(plans, gdev)]
    with mlba.Batch(plans, max_iters=iters) as batch:
        outs, _ = batch.restore(gdev, alpha=alpha, mu=1e-3, delta=delta, iters=iters, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(outs[i], ref[i]), i
        got = host(outs[1])
    want = omlba.mlba(gs[1], Hs[1], AR_BC, opc.AR, 2, np.full(iters, alpha), np.full(iters + 1, delta), 1e-3,
                      iters)["f"]
    assert rel_err(got, want) < 1e-4
    for pl in plans:
        pl.close()
