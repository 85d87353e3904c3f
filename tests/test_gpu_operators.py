"""Per-operator parity of the HIP library against the FP64 oracle.

Each operator is called through the C ABI (python binding = marshalling) on
seeded inputs and compared element by element with the oracle.  Bar:
||gpu - oracle||_2 / ||oracle||_2 <= 1e-5 and max |gpu - oracle| <= 1e-4 max
|oracle| per operator (float32 arithmetic against float64).
"""
import numpy as np
import pytest

import synth
from oracle import blur as oblur
from oracle import framelet as ofr
from oracle import mlba as omlba
from oracle import precond as opc
from tests._util import announce, cuda, host, max_err, rel_err

pytestmark = pytest.mark.gpu

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
    if kind == "disk":
        return synth.disk_psf(p, (p - 1) / 2.0)
    h = g.random((p, p))
    return h / h.sum()


BLUR_CASES = [
    # (n, p, psf kind)   n not a multiple of the tile, p across the template range and the generic path
    (64, 9, "gauss"),
    (100, 7, "rand"),
    (96, 17, "motion"),
    (150, 31, "disk"),
    (77, 35, "rand"),
    (33, 1, "rand"),
]


@pytest.mark.parametrize("bc", [0, 1, 2, 3])
@pytest.mark.parametrize("n,p,kind", BLUR_CASES)
def test_blur_and_transpose(mlba, bc, n, p, kind):
    announce(f"blur bc={bc} n={n} p={p} {kind}")
    H = _psf(kind, p, n + p)
    g = synth.rng(1000 + n * 3 + p + bc)
    N = oblur.unknown_side(n, p, bc)
    u = g.random((N, N))
    y = g.standard_normal((n, n))
    gi = g.random((n, n))
    with mlba.Plan(n, p, bc, mlba.NONE, 1, cuda(H)) as plan:
        Au = host(plan.apply_A(cuda(u)))
        Aty = host(plan.apply_At(cuda(y)))
        r = host(plan.residual(cuda(gi), cuda(u)))
    ref_Au = oblur.blur(u, H, bc, "direct" if n <= 100 else "fft")
    ref_Aty = oblur.blurT(y, H, bc, "direct" if n <= 100 else "fft")
    assert rel_err(Au, ref_Au) < TOL_L2 and max_err(Au, ref_Au) < TOL_MAX
    assert rel_err(Aty, ref_Aty) < TOL_L2 and max_err(Aty, ref_Aty) < TOL_MAX
    assert rel_err(r, gi - ref_Au) < TOL_L2
    # adjoint identity of the GPU pair, evaluated in float64
    lhs, rhs = np.vdot(Au, y), np.vdot(u, Aty)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Au) * np.linalg.norm(y)


# 14, 196, 998 have a prime factor >= 7: Bluestein form over m = 27, 400, 2000
@pytest.mark.parametrize("n", [8, 10, 14, 64, 96, 100, 192, 196, 250, 256, 384, 512, 768, 998, 1000, 1024, 2000,
                               2048])
@pytest.mark.parametrize("pc", [0, 1])
def test_preconditioner(mlba, n, pc):
    p = 9 if n >= 9 else 3
    announce(f"precond pc={pc} n={n} p={p}")
    H = _psf("motion" if n >= 64 else "rand", p, n)
    g = synth.rng(2000 + n + pc)
    smooth = synth.shapes_image(n, g, n_rect=6, n_disk=3, n_bumps=3)
    noise = g.standard_normal((n, n))
    with mlba.Plan(n, p, 0, pc, 1, cuda(H)) as plan:
        for alpha in (0.5, 0.05, 0.02):
            for r in (smooth, noise):
                got = host(plan.apply_P(cuda(r), alpha))
                ref = opc.apply(r, H, alpha, pc)
                e2, em = rel_err(got, ref), max_err(got, ref)
                print(f"  alpha={alpha} l2={e2:.2e} max={em:.2e}", flush=True)
                assert e2 < TOL_L2 and em < TOL_MAX


def test_preconditioner_in_place(mlba):
    n, p = 128, 7
    announce("precond in place")
    H = _psf("rand", p, 5)
    r = synth.rng(5).standard_normal((n, n))
    with mlba.Plan(n, p, 0, 0, 1, cuda(H)) as plan:
        t = cuda(r)
        plan.apply_P(t, 0.1, out=t)
        assert rel_err(host(t), opc.apply_bccb(r, H, 0.1)) < TOL_L2


FRAME_CASES = [(9, 1), (72, 1), (104, 2), (257, 3), (300, 4), (528, 2), (130, 4)]


@pytest.mark.parametrize("N,L", FRAME_CASES)
def test_framelet(mlba, N, L):
    announce(f"framelet N={N} L={L}")
    g = synth.rng(3000 + N + L)
    f = synth.shapes_image(N, g, n_rect=8, n_disk=4, n_bumps=4)
    # a plan whose unknown side is N: periodic boundary, n = N, no preconditioner
    with mlba.Plan(N, 1, 2, mlba.NONE, L, cuda(np.ones((1, 1)))) as plan:
        assert plan.N == N and plan.bands == 8 * L + 1
        z = plan.analysis(cuda(f))
        zr = ofr.analysis(f, L)
        assert rel_err(host(z), zr) < TOL_L2 and max_err(host(z), zr) < TOL_MAX
        zz = g.standard_normal(zr.shape)
        s = host(plan.synthesis(cuda(zz)))
        sr = ofr.synthesis(zz, L)
        assert rel_err(s, sr) < TOL_L2 and max_err(s, sr) < TOL_MAX
        mu = np.linspace(0.05, 0.6, 8 * L + 1)
        ts = host(plan.threshold_synthesis(cuda(zz), mu, 0.7))
        tr = ofr.synthesis(0.7 * omlba.soft_threshold(zz, mu), L)
        assert rel_err(ts, tr) < TOL_L2 and max_err(ts, tr) < TOL_MAX
        z0 = cuda(zz)
        w = g.standard_normal((N, N))
        plan.analysis_update(cuda(w), z0)
        ur = zz + ofr.analysis(w, L)
        assert rel_err(host(z0), ur) < TOL_L2
        # perfect reconstruction of the GPU pair
        assert rel_err(host(plan.synthesis(z)), f) < TOL_L2


def test_soft_threshold(mlba):
    announce("soft threshold")
    g = synth.rng(4)
    z = g.standard_normal((17, 33, 31))
    mu = np.linspace(0, 1.5, 17)
    got = host(mlba.soft_threshold(cuda(z), mu, 0.8))
    ref = 0.8 * omlba.soft_threshold(z, mu)
    assert np.abs(got - ref).max() < 1e-6
    x = np.array([[-3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 3.0, 1.25]])
    assert np.array_equal(host(mlba.soft_threshold(cuda(x), 1.0, 1.0))[0], [-2.0, 0, 0, 0, 0, 0, 2.0, 0.25])


@pytest.mark.parametrize("n,psf,bc,pc,alpha", [
    (64, "gauss9", 0, 0, 0.05), (64, "gauss9", 1, 1, 0.05), (64, "gauss9", 0, 1, 0.05),
    (96, "gauss9", 2, 0, 0.1), (96, "gauss9", 3, 1, 0.2), (80, "motion17", 0, 2, 1.0),
    (256, "disk31", 0, 0, 0.02), (256, "motion17", 1, 1, 0.05)])
def test_opnorm(mlba, n, psf, bc, pc, alpha):
    """||A^T P_alpha A|| (the norm of section 3's step rule) by Lanczos on the GPU
    against the oracle's ARPACK value converged in FP64; the motion-blur
    reflective case has clustered top eigenvalues (slow convergence)."""
    announce(f"opnorm n={n} psf={psf} bc={bc} pc={pc} alpha={alpha}")
    H = {"gauss9": lambda: synth.gaussian_psf(9, 2.0), "disk31": lambda: synth.disk_psf(31, 15.0),
         "motion17": lambda: synth.motion_psf(17, 15.0, 0.7)}[psf]()
    with mlba.Plan(n, H.shape[0], bc, pc, 1, cuda(H)) as plan:
        got = plan.opnorm(alpha)
    ref = omlba.opnorm(H, n, bc, pc, alpha, tol=1e-12)
    print(f"  gpu={got:.9f} oracle={ref:.9f} rel {abs(got / ref - 1):.1e}", flush=True)
    assert abs(got / ref - 1.0) <= 1e-6


@pytest.mark.parametrize("n,bc,pc,alpha", [(96, 1, 0, 0.05), (96, 2, 0, 0.1), (96, 3, 1, 0.2), (256, 1, 1, 0.05),
                                         (256, 0, 0, 0.02)])
def test_opnorm_fft_blur(mlba, n, bc, pc, alpha):
    """The same norm with A and A^T on the FFT grid (the square models' pad
    placed on the grid and folded back by its transpose): against the oracle
    and against the direct blur's Lanczos."""
    announce(f"opnorm FFT blur n={n} bc={bc} pc={pc} alpha={alpha}")
    H = synth.motion_psf(17, 15.0, 0.7) if n == 256 else synth.gaussian_psf(9, 2.0)
    with mlba.Plan(n, H.shape[0], bc, pc, 1, cuda(H)) as plan:
        direct = plan.opnorm(alpha)
        plan.set_blur(mlba.BLUR_FFT)
        got = plan.opnorm(alpha)
    ref = omlba.opnorm(H, n, bc, pc, alpha, tol=1e-12)
    print(f"  fft={got:.9f} direct={direct:.9f} oracle={ref:.9f} rel {abs(got / ref - 1):.1e}", flush=True)
    assert abs(got / ref - 1.0) <= 1e-6
    assert abs(got / direct - 1.0) <= 1e-6


def test_full_size_operators(mlba):
    """The 2048 x 2048 throughput workload's shapes: p = 31 disk, 3 levels."""
    w = synth.make_workload("rect-bccb-2048")
    announce("full size operators n=2048 p=31 L=3")
    u = w.truth
    with mlba.Plan(w.n, w.p, 0, 0, 3, cuda(w.psf)) as plan:
        Au = host(plan.apply_A(cuda(u)))
        ref = oblur.blur_fft(u, w.psf, 0)
        assert rel_err(Au, ref) < TOL_L2
        P_ = host(plan.apply_P(cuda(Au), w.alpha0))
        refP = opc.apply_bccb(Au, w.psf, w.alpha0)
        print(f"  P fp32 error l2={rel_err(P_, refP):.2e}", flush=True)
        assert rel_err(P_, refP) < TOL_L2
        At = host(plan.apply_At(cuda(refP)))
        assert rel_err(At, oblur.blurT_fft(refP, w.psf, 0)) < TOL_L2
        z = host(plan.analysis(cuda(u)))
        assert rel_err(z, ofr.analysis(u, 3)) < TOL_L2
