"""Pins of the FP64 oracle to facts fixed outside the oracle itself.

Each test checks the oracle against a library routine, a closed form, an
invariant stated by the paper, a brute-force dense computation on a tiny
problem, or the worked matrices printed in section 6.1.  None of them needs a
GPU.
"""
import math
import os

import numpy as np
import pytest
import scipy.fft
import scipy.ndimage
import scipy.signal

import synth
from oracle import blur, framelet, mlba, precond

RECT, REFLECT, PERIODIC, ZERO = blur.RECT, blur.REFLECT, blur.PERIODIC, blur.ZERO
BCCB, DCT, NONE = precond.BCCB, precond.DCT, precond.NONE
ND_MODE = {REFLECT: "reflect", PERIODIC: "wrap", ZERO: "constant"}


def rand_psf(g, p, sym=False):
    h = g.random((p, p))
    if sym:
        h = h + h[::-1, :] + h[:, ::-1] + h[::-1, ::-1]
    return h / h.sum()


def dense_of(op, shape_in):
    """Columns of op applied to unit images (brute force matrix)."""
    k = int(np.prod(shape_in))
    cols = []
    for i in range(k):
        e = np.zeros(k)
        e[i] = 1.0
        cols.append(np.asarray(op(e.reshape(shape_in))).ravel())
    return np.stack(cols, axis=1)


# ---------------------------------------------------------------------------
# blur A (section 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,p", [(8, 3), (13, 5), (20, 7), (31, 9)])
def test_rect_blur_is_scipy_valid_convolution(n, p):
    g = synth.rng(n * 10 + p)
    H = rand_psf(g, p)
    f = g.standard_normal((n + p - 1, n + p - 1))
    ref = scipy.signal.convolve2d(f, H, mode="valid")
    assert np.allclose(blur.blur_direct(f, H, RECT), ref, atol=1e-13, rtol=0)
    # A^T is MATLAB's conv2(y, rot90(H, 2), 'full')
    y = g.standard_normal((n, n))
    refT = scipy.signal.convolve2d(y, H[::-1, ::-1], mode="full")
    assert np.allclose(blur.blurT_direct(y, H, RECT), refT, atol=1e-13, rtol=0)


@pytest.mark.parametrize("bc", [REFLECT, PERIODIC, ZERO])
@pytest.mark.parametrize("n,p", [(8, 3), (12, 5), (17, 7)])
def test_bc_blur_is_scipy_ndimage_convolution(bc, n, p):
    """Table 1 padding: scipy.ndimage's 'reflect' (half-sample symmetric),
    'wrap' and zero 'constant' modes with a centred odd kernel."""
    g = synth.rng(100 + n * 10 + p + bc)
    H = rand_psf(g, p)
    f = g.standard_normal((n, n))
    ref = scipy.ndimage.convolve(f, H, mode=ND_MODE[bc], cval=0.0)
    assert np.allclose(blur.blur_direct(f, H, bc), ref, atol=1e-13, rtol=0)


@pytest.mark.parametrize("bc", [RECT, REFLECT, PERIODIC, ZERO])
def test_blur_fft_matches_direct(bc):
    g = synth.rng(7 + bc)
    n, p = 40, 9
    H = rand_psf(g, p)
    N = blur.unknown_side(n, p, bc)
    f = g.standard_normal((N, N))
    y = g.standard_normal((n, n))
    assert np.abs(blur.blur_fft(f, H, bc) - blur.blur_direct(f, H, bc)).max() < 1e-13
    assert np.abs(blur.blurT_fft(y, H, bc) - blur.blurT_direct(y, H, bc)).max() < 1e-13


@pytest.mark.parametrize("bc", [RECT, REFLECT, PERIODIC, ZERO])
@pytest.mark.parametrize("method", ["direct", "fft"])
def test_blur_adjoint_identity(bc, method):
    g = synth.rng(11 + bc)
    n, p = 24, 7
    H = rand_psf(g, p)
    N = blur.unknown_side(n, p, bc)
    x = g.standard_normal((N, N))
    y = g.standard_normal((n, n))
    lhs = np.vdot(blur.blur(x, H, bc, method), y)
    rhs = np.vdot(x, blur.blurT(y, H, bc, method))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def test_blur_transpose_is_dense_transpose():
    g = synth.rng(3)
    n, p = 5, 3
    H = rand_psf(g, p)
    for bc in (RECT, REFLECT, PERIODIC, ZERO):
        N = blur.unknown_side(n, p, bc)
        Ad = dense_of(lambda f: blur.blur_direct(f, H, bc), (N, N))
        Atd = dense_of(lambda y: blur.blurT_direct(y, H, bc), (n, n))
        assert np.abs(Ad.T - Atd).max() < 1e-15


def test_blur_norm_at_most_one():
    """Nonnegative PSF of sum one: the largest singular value of A is <= 1
    (section 4.2, the spectrum of A A^T + alpha I lies in [alpha, 1 + alpha])."""
    g = synth.rng(5)
    n, p = 6, 3
    H = rand_psf(g, p)
    for bc in (RECT, PERIODIC, ZERO):
        N = blur.unknown_side(n, p, bc)
        Ad = dense_of(lambda f: blur.blur_direct(f, H, bc), (N, N))
        assert np.linalg.norm(Ad, 2) <= 1 + 1e-12
    # mirrored borders count a pixel twice: the bound needs a symmetric PSF
    Hs = rand_psf(g, p, sym=True)
    Ad = dense_of(lambda f: blur.blur_direct(f, Hs, REFLECT), (n, n))
    assert abs(np.linalg.norm(Ad, 2) - 1.0) < 1e-12
    # periodic: exactly 1 (constants are preserved)
    N = n
    Ad = dense_of(lambda f: blur.blur_direct(f, H, PERIODIC), (N, N))
    assert abs(np.linalg.norm(Ad, 2) - 1.0) < 1e-12


def test_valid_blur_is_interior_of_periodic_blur():
    """Section 2.1: A = M A_big with A_big the m x m BCCB blur."""
    g = synth.rng(9)
    n, p = 16, 5
    c = (p - 1) // 2
    H = rand_psf(g, p)
    f = g.standard_normal((n + p - 1, n + p - 1))
    big = blur.blur_direct(f, H, PERIODIC)
    assert np.abs(blur.blur_direct(f, H, RECT) - big[c:c + n, c:c + n]).max() < 1e-14


# ---------------------------------------------------------------------------
# framelet W (section 6.1)
# ---------------------------------------------------------------------------

def _read_printed(golden_dir):
    mats, name, rows = {}, None, []
    with open(os.path.join(golden_dir, "framelet_printed_1d.txt")) as fh:
        for line in fh:
            s = line.strip()
            if not s or s.startswith("#"):
                continue
            if s[0].isalpha():
                if name:
                    mats[name] = np.array(rows, dtype=float) / 4.0
                name, rows = s, []
            else:
                rows.append([float(t) for t in s.split()])
    mats[name] = np.array(rows, dtype=float) / 4.0
    return mats


def test_printed_framelet_matrices(golden_dir):
    m = _read_printed(golden_dir)
    N = m["B0"].shape[0]
    assert np.allclose(framelet.dense_1d(0, N), m["B0"], atol=1e-15)
    # printed "B1" is the mask b2; printed "B2" is b1 / sqrt(2)
    assert np.allclose(framelet.dense_1d(2, N), m["B1"], atol=1e-15)
    assert np.allclose(framelet.dense_1d(1, N), math.sqrt(2) * m["B2"], atol=1e-15)
    # the printed B2 without sqrt(2) is not a tight frame, the masks are
    printed = [m["B0"], m["B1"], m["B2"]]
    assert np.abs(sum(b.T @ b for b in printed) - np.eye(N)).max() > 0.1
    masks = [framelet.dense_1d(i, N) for i in range(3)]
    assert np.abs(sum(b.T @ b for b in masks) - np.eye(N)).max() < 1e-15


@pytest.mark.parametrize("N", [5, 8, 13, 32])
def test_one_level_is_kronecker_stack(N):
    """W = [B_00; B_01; ...; B_22] with B_ij = B_i (x) B_j acting on the
    column-stacked image (section 6.1, section 1 stack ordering)."""
    g = synth.rng(N)
    f = g.standard_normal((N, N))
    z = framelet.analysis(f, 1)
    vec = f.ravel(order="F")
    D = [framelet.dense_1d(i, N) for i in range(3)]
    for (i, j), b in [((0, 0), 0)] + [(pq, 1 + q) for q, pq in enumerate(framelet.PAIRS)]:
        ref = (np.kron(D[i], D[j]) @ vec).reshape((N, N), order="F")
        assert np.abs(z[b] - ref).max() < 1e-13


@pytest.mark.parametrize("N", [7, 16, 33, 64])
@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_framelet_perfect_reconstruction(N, L):
    """W^T W = I (section 1, eq. wavecoeff; section 3)."""
    if 2 ** (L - 1) > N:
        pytest.skip("dilation larger than the image")
    g = synth.rng(N * 7 + L)
    f = g.standard_normal((N, N))
    z = framelet.analysis(f, L)
    assert z.shape == (8 * L + 1, N, N)
    assert np.abs(framelet.synthesis(z, L) - f).max() < 1e-13
    assert abs(np.linalg.norm(z) - np.linalg.norm(f)) < 1e-12 * np.linalg.norm(f)
    zz = g.standard_normal(z.shape)
    lhs, rhs = np.vdot(z, zz), np.vdot(f, framelet.synthesis(zz, L))
    assert abs(lhs - rhs) < 1e-12 * max(1, abs(lhs))


def test_framelet_dense_tight_frame_small():
    """Brute force: the dense W of a 6 x 6 image, 2 levels, has W^T W = I and
    W W^T a projection (not the identity)."""
    N, L = 6, 2
    Wd = dense_of(lambda f: framelet.analysis(f, L), (N, N))
    assert np.abs(Wd.T @ Wd - np.eye(N * N)).max() < 1e-14
    P = Wd @ Wd.T
    assert np.abs(P @ P - P).max() < 1e-14
    assert np.abs(P - np.eye(P.shape[0])).max() > 0.1


def test_framelet_constant_image():
    """Masks b1, b2 sum to zero and the reflective extension of a constant is
    constant: only the low-pass band survives, at every level."""
    N, L = 20, 3
    z = framelet.analysis(np.full((N, N), 2.5), L)
    assert np.abs(z[0] - 2.5).max() < 1e-14
    assert np.abs(z[1:]).max() < 1e-14


def test_band_axes_convention():
    """An image varying only along x leaves bands with a high-pass filter
    along y (j != 0) empty; the x-high-pass bands (i != 0, j = 0) are not."""
    N = 24
    x = np.arange(N, dtype=float)
    f = np.tile(np.sin(0.7 * x) + 0.01 * x * x, (N, 1))
    z = framelet.analysis(f, 1)
    for q, (i, j) in enumerate(framelet.PAIRS):
        if j != 0:
            assert np.abs(z[1 + q]).max() < 1e-13
        else:
            assert np.abs(z[1 + q]).max() > 1e-3


# ---------------------------------------------------------------------------
# preconditioners (Algorithms 1 and 3)
# ---------------------------------------------------------------------------

def _dense_bc_blur(H, n, mode):
    return dense_of(lambda f: scipy.ndimage.convolve(f, H, mode=mode, cval=0.0), (n, n))


@pytest.mark.parametrize("p", [3, 5, 7])
@pytest.mark.parametrize("alpha", [0.5, 0.05, 1e-3])
def test_bccb_preconditioner_is_dense_solve(p, alpha):
    n = 8
    g = synth.rng(p * 100 + int(alpha * 1e4))
    H = rand_psf(g, p)
    C = _dense_bc_blur(H, n, "wrap")
    r = g.standard_normal((n, n))
    ref = np.linalg.solve(C @ C.T + alpha * np.eye(n * n), r.ravel()).reshape(n, n)
    got = precond.apply_bccb(r, H, alpha)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("p", [3, 5, 7])
@pytest.mark.parametrize("alpha", [0.5, 0.05, 1e-3])
def test_dct_preconditioner_is_dense_solve(p, alpha):
    """Algorithm 3: Q is the reflective-boundary blur of the symmetrised PSF."""
    n = 8
    g = synth.rng(p * 1000 + int(alpha * 1e4))
    H = rand_psf(g, p)
    Q = _dense_bc_blur(precond.symmetrize(H), n, "reflect")
    r = g.standard_normal((n, n))
    ref = np.linalg.solve(Q @ Q.T + alpha * np.eye(n * n), r.ravel()).reshape(n, n)
    got = precond.apply_dct(r, H, alpha)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n,p", [(8, 3), (10, 5), (12, 7)])
def test_dct_eigen_pairs(n, p):
    """Q v = lambda v for every 2-D DCT-II basis image v (reflective blur of a
    quadrantally symmetric PSF)."""
    g = synth.rng(n + p)
    Hs = rand_psf(g, p, sym=True)
    Q = _dense_bc_blur(Hs, n, "reflect")
    lam = precond.dct_eigs(Hs, n)
    for k in range(n):
        for l in range(n):
            e = np.zeros((n, n))
            e[k, l] = 1.0
            v = scipy.fft.idctn(e, type=2, norm="ortho")
            assert np.abs(Q @ v.ravel() - lam[k, l] * v.ravel()).max() < 1e-13


def test_library_transforms_match_naive():
    """The FFT and orthonormal DCT-II routines the oracle calls agree with the
    O(N^2) sums that define them."""
    g = synth.rng(21)
    N = 12
    x = g.standard_normal(N)
    j = np.arange(N)
    F = np.exp(-2j * np.pi * np.outer(j, j) / N)
    assert np.abs(np.fft.fft(x) - F @ x).max() < 1e-12
    Cd = np.sqrt(2.0 / N) * np.cos(np.pi * np.outer(j, 2 * j + 1) / (2 * N))
    Cd[0] /= np.sqrt(2.0)
    assert np.abs(scipy.fft.dct(x, type=2, norm="ortho") - Cd @ x).max() < 1e-12
    assert np.abs(Cd @ Cd.T - np.eye(N)).max() < 1e-13


def test_symmetrize():
    g = synth.rng(31)
    p = 7
    Hs = rand_psf(g, p, sym=True)
    assert np.abs(precond.symmetrize(Hs) - Hs).max() < 1e-16
    H = rand_psf(g, p)
    Ht = precond.symmetrize(H)
    assert abs(Ht.sum() - 1.0) < 1e-14
    # Frobenius-optimal: H - H~ is orthogonal to every quadrantally symmetric S
    for _ in range(5):
        q = g.standard_normal((4, 4))
        S = np.zeros((p, p))
        S[3:, 3:] = q
        S[:3, 3:] = q[1:][::-1]
        S[3:, :3] = q[:, 1:][:, ::-1]
        S[:3, :3] = q[1:, 1:][::-1, ::-1]
        assert np.abs(S - S[::-1] ).max() < 1e-16 and np.abs(S - S[:, ::-1]).max() < 1e-16
        assert abs(np.vdot(H - Ht, S)) < 1e-14


def test_bccb_spectrum_in_unit_interval():
    g = synth.rng(41)
    H = rand_psf(g, 9)
    s = precond.bccb_eigs_sq(H, 32)
    assert s.min() >= 0 and s.max() <= 1 + 1e-14
    assert abs(s[0, 0] - 1.0) < 1e-14


# ---------------------------------------------------------------------------
# soft threshold (eq. soft)
# ---------------------------------------------------------------------------

def test_soft_threshold_closed_form():
    x = np.array([-3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 3.0, 1.25])
    assert np.array_equal(mlba.soft_threshold(x, 1.0), [-2.0, 0, 0, 0, 0, 0, 2.0, 0.25])
    assert np.array_equal(mlba.soft_threshold(x, 0.0), x)
    z = np.ones((3, 2, 2)) * np.array([1.0, 2.0, 3.0])[:, None, None]
    out = mlba.soft_threshold(z, np.array([0.5, 2.0, 4.0]))
    assert np.array_equal(out[:, 0, 0], [0.5, 0.0, 0.0])


# ---------------------------------------------------------------------------
# the iteration (section 3, eq. MLBA2)
# ---------------------------------------------------------------------------

def _small_problem(seed, n=12, p=5, bc=RECT, noise=0.01):
    g = synth.rng(seed)
    H = rand_psf(g, p)
    m = n + p - 1
    truth = synth.shapes_image(m, g, n_rect=4, n_disk=2)
    gimg = synth.add_noise(blur.blur_direct(truth, H, RECT), synth.white_noise((n, n), g), noise)
    if bc != RECT:
        c = (p - 1) // 2
        truth = truth[c:c + n, c:c + n]
    return gimg, H, truth


@pytest.mark.parametrize("bc,pc", [(RECT, BCCB), (RECT, DCT), (REFLECT, DCT), (ZERO, BCCB)])
def test_mu_zero_is_preconditioned_landweber(bc, pc):
    """With mu = 0 the threshold is the identity and W^T W = I, so W^T x^k
    follows f^{k+1} = f^k + delta A^T P (g - A f^k)."""
    gimg, H, _ = _small_problem(1 + bc + 10 * pc, bc=bc)
    L, K, alpha, delta = 2, 15, 0.1, 0.5
    out = mlba.mlba(gimg, H, bc, pc, L, np.full(K, alpha), np.full(K + 1, delta), 0.0, K)
    N = out["f"].shape[0]
    f = np.zeros((N, N))
    for _ in range(K):
        f = f + delta * blur.blurT(precond.apply(gimg - blur.blur(f, H, bc), H, alpha, pc), H, bc)
    assert np.abs(out["f"] - f).max() < 1e-12 * max(1, np.abs(f).max())


def test_periodic_landweber_closed_form():
    """Periodic boundary + BCCB preconditioner + mu = 0: in the Fourier domain
    f^K = (1 - rho^K) g / Lambda with rho = 1 - delta |Lambda|^2/(|Lambda|^2 + alpha),
    Lambda the DFT of the first column of the circulant A."""
    n, p = 16, 5
    g = synth.rng(77)
    H = rand_psf(g, p)
    gimg = g.standard_normal((n, n))
    e0 = np.zeros((n, n))
    e0[0, 0] = 1.0
    lam = np.fft.fft2(blur.blur_direct(e0, H, PERIODIC))
    assert np.abs(lam).min() > 1e-8
    for K in (1, 7, 40):
        for alpha, delta in ((0.05, 0.3), (0.5, 1.0)):
            out = mlba.mlba(gimg, H, PERIODIC, BCCB, 1, np.full(K, alpha), np.full(K + 1, delta), 0.0, K)
            s = np.abs(lam) ** 2
            rho = 1.0 - delta * s / (s + alpha)
            ref = np.fft.ifft2((1.0 - rho ** K) * np.fft.fft2(gimg) / lam).real
            assert np.abs(out["f"] - ref).max() < 1e-11 * max(1, np.abs(ref).max())


def _dense_ops(H, n, bc, L):
    p = H.shape[0]
    N = blur.unknown_side(n, p, bc)
    B = framelet.n_bands(L)
    Ad = dense_of(lambda f: blur.blur_direct(f, H, bc), (N, N))
    Wd = dense_of(lambda f: framelet.analysis(f, L), (N, N))
    return Ad, Wd, N, B


def _lbi(K, g, mu, lam, iters, B, N):
    """eq. (iterLinBreg) on dense matrices."""
    z = np.zeros(K.shape[1])
    x = np.zeros_like(z)
    mu_full = np.repeat(np.broadcast_to(mu, (B,)), N * N)
    for _ in range(iters):
        z = z + K.T @ (g - K @ x)
        x = lam * np.sign(z) * np.maximum(np.abs(z) - mu_full, 0.0)
    return z, x


def test_identity_preconditioner_is_linearized_bregman():
    gimg, H, _ = _small_problem(5, n=6, p=3)
    L, iters, lam = 1, 12, 0.8
    mu = 0.02
    Ad, Wd, N, B = _dense_ops(H, 6, RECT, L)
    K = Ad @ Wd.T
    z_ref, x_ref = _lbi(K, gimg.ravel(), mu, lam, iters, B, N)
    out = mlba.mlba(gimg, H, RECT, NONE, L, np.zeros(iters), np.full(iters + 1, lam), mu, iters)
    assert np.abs(out["z"].ravel() - z_ref).max() < 1e-12
    assert np.abs(out["f"].ravel() - Wd.T @ x_ref).max() < 1e-12


@pytest.mark.parametrize("pc", [BCCB, DCT])
def test_mlba_is_lbi_on_preconditioned_system(pc):
    """Remark (rem:prec): MLBA with P is LBI for P^{1/2} K x = P^{1/2} g."""
    n, p = 6, 3
    gimg, H, _ = _small_problem(9 + pc, n=n, p=p)
    L, iters, lam, alpha, mu = 1, 10, 0.25, 0.1, 0.01
    Ad, Wd, N, B = _dense_ops(H, n, RECT, L)
    if pc == BCCB:
        C = _dense_bc_blur(H, n, "wrap")
    else:
        C = _dense_bc_blur(precond.symmetrize(H), n, "reflect")
    P = np.linalg.inv(C @ C.T + alpha * np.eye(n * n))
    w, V = np.linalg.eigh(P)
    Ph = V @ np.diag(np.sqrt(w)) @ V.T
    z_ref, x_ref = _lbi(Ph @ Ad @ Wd.T, Ph @ gimg.ravel(), mu, lam, iters, B, N)
    out = mlba.mlba(gimg, H, RECT, pc, L, np.full(iters, alpha), np.full(iters + 1, lam), mu, iters)
    assert np.abs(out["z"].ravel() - z_ref).max() < 1e-11
    assert np.abs(out["f"].ravel() - Wd.T @ x_ref).max() < 1e-11


def test_state_stays_in_range_of_W():
    """z^k is a sum of W(.) terms, so W W^T z^k = z^k."""
    gimg, H, _ = _small_problem(13, n=20, p=5)
    L = 2
    out = mlba.mlba(gimg, H, RECT, BCCB, L, np.full(8, 0.1), np.full(9, 0.3), 1e-3, 8)
    z = out["z"]
    assert np.abs(framelet.analysis(framelet.synthesis(z, L), L) - z).max() < 1e-12 * np.abs(z).max()


def test_resume_equals_uninterrupted():
    gimg, H, _ = _small_problem(17, n=16, p=5)
    al, de = np.full(12, 0.1), np.full(13, 0.3)
    full = mlba.mlba(gimg, H, RECT, BCCB, 2, al, de, 1e-3, 12)
    half = mlba.mlba(gimg, H, RECT, BCCB, 2, al, de, 1e-3, 5)
    rest = mlba.mlba(gimg, H, RECT, BCCB, 2, al, de, 1e-3, 7, z0=half["z"], k0=5)
    assert np.array_equal(rest["z"], full["z"])
    assert np.array_equal(np.concatenate([half["rnorm"], rest["rnorm"]]), full["rnorm"])


def test_opnorm_matches_dense():
    n, p = 6, 3
    g = synth.rng(23)
    H = rand_psf(g, p)
    for bc, pc in ((RECT, BCCB), (REFLECT, DCT), (RECT, DCT)):
        N = blur.unknown_side(n, p, bc)
        Ad = dense_of(lambda f: blur.blur_direct(f, H, bc), (N, N))
        Pd = dense_of(lambda r: precond.apply(r, H, 0.05, pc), (n, n))
        ref = np.linalg.eigvalsh(Ad.T @ Pd @ Ad).max()
        assert abs(mlba.opnorm(H, n, bc, pc, 0.05) - ref) < 1e-8 * ref


def test_converges_to_noise_level_with_auto_step():
    """Theorem (MLBA convergence) for delta < 1/||A^T P A||: the residual
    falls to the order of the noise norm and stays finite."""
    w = synth.make_workload("plain-fp64-72")
    gimg = synth.add_noise(blur.blur(w.truth, w.psf, RECT), w.xi, w.noise_level)
    nn = synth.noise_norm(blur.blur(w.truth, w.psf, RECT), w.noise_level)
    d = mlba.delta_auto(mlba.opnorm(w.psf, w.n, RECT, BCCB, w.alpha0))
    out = mlba.mlba(gimg, w.psf, RECT, BCCB, 1, np.full(50, w.alpha0), np.full(51, d), w.mu, 50)
    r = out["rnorm"]
    assert np.all(np.isfinite(r))
    assert r[-1] < 1.5 * nn and r[-1] < 0.05 * r[0]


def test_literal_unit_step_diverges():
    """The 72 x 72 workload with the literal step 1: ||A^T P A|| > 1 at
    alpha = 0.05, so the iteration is outside the convergence theorem and
    the residual grows without bound."""
    w = synth.make_workload("plain-fp64-72")
    gimg = synth.add_noise(blur.blur(w.truth, w.psf, RECT), w.xi, w.noise_level)
    assert mlba.opnorm(w.psf, w.n, RECT, BCCB, w.alpha0) > 1.0
    out = mlba.mlba(gimg, w.psf, RECT, BCCB, 1, np.full(50, w.alpha0), np.full(51, 1.0), w.mu, 50)
    assert out["rnorm"][-1] > 1e3 * out["rnorm"][0]


def test_alpha_table():
    """The geometric schedule (reading R9) against its recursive form
    a_{k+1} = max(r a_k, floor) and the index where the floor takes over,
    ceil(log(floor / a_0) / log r); the constant schedule."""
    a0, r, floor, K = 0.5, 0.8, 0.02, 30
    a = mlba.alpha_table(1, a0, K, ratio=r, floor=floor)
    rec = [a0]
    for _ in range(K - 1):
        rec.append(max(rec[-1] * r, floor))
    assert np.allclose(a, rec, rtol=1e-13, atol=0.0)
    k_floor = int(np.ceil(np.log(floor / a0) / np.log(r)))
    assert np.all(a[:k_floor] > floor) and np.all(a[k_floor:] == floor)
    assert np.all(np.diff(a) <= 0.0)
    assert np.all(mlba.alpha_table(0, 0.05, 4) == 0.05)
