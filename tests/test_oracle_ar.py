"""Pins of the oracle's antireflective model (sections 2.2 and 4.3) to facts
fixed outside it: the paper's pixel formulas for the edges and corners of the
pad, the affine images the antireflective extension preserves, the paper's
remark that the reblurring matrix equals A^T for zero and periodic
conditions, and brute-force dense matrices on tiny problems for the
transform, the preconditioner, the Algorithm 4 direction, the operator norm
and a threshold-free run.  None of them needs a GPU.
"""
import numpy as np
import pytest

import synth
from oracle import alg4, blur, mlba, precond

AR = blur.ANTIREFLECT


def rand_psf(g, p, sym=False):
    h = g.random((p, p))
    if sym:
        h = h + h[::-1, :] + h[:, ::-1] + h[::-1, ::-1]
    return h / h.sum()


def dense_of(op, n):
    cols = []
    for i in range(n * n):
        e = np.zeros(n * n)
        e[i] = 1.0
        cols.append(np.asarray(op(e.reshape(n, n))).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("n,c", [(7, 3), (5, 4), (12, 2), (6, 1)])
def test_pad_matches_the_papers_edge_and_corner_formulas(n, c):
    """Section 2.2 prints the pad pixel by pixel in 1-based indices:
    F(1-i, j) = 2F(1, j) - F(i+1, j) and its three companions on the edges,
    F(1-i, 1-j) = 4F(1,1) - 2F(1, j+1) - 2F(i+1, 1) + F(i+1, j+1) and its
    companions in the corners.  They are written out here one by one."""
    F1 = synth.rng(n + 31 * c).standard_normal((n, n))

    def F(i, j):  # 1-based access
        return F1[i - 1, j - 1]

    ref = {}
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            ref[i, j] = F(i, j)
    for i in range(1, c + 1):
        for j in range(1, n + 1):
            ref[1 - i, j] = 2 * F(1, j) - F(i + 1, j)
            ref[n + i, j] = 2 * F(n, j) - F(n - i, j)
            ref[j, 1 - i] = 2 * F(j, 1) - F(j, i + 1)
            ref[j, n + i] = 2 * F(j, n) - F(j, n - i)
    for i in range(1, c + 1):
        for j in range(1, c + 1):
            ref[1 - i, 1 - j] = 4 * F(1, 1) - 2 * F(1, j + 1) - 2 * F(i + 1, 1) + F(i + 1, j + 1)
            ref[1 - i, n + j] = 4 * F(1, n) - 2 * F(1, n - j) - 2 * F(i + 1, n) + F(i + 1, n - j)
            ref[n + i, 1 - j] = 4 * F(n, 1) - 2 * F(n, j + 1) - 2 * F(n - i, 1) + F(n - i, j + 1)
            ref[n + i, n + j] = 4 * F(n, n) - 2 * F(n, n - j) - 2 * F(n - i, n) + F(n - i, n - j)
    pad = blur._extend(F1, c, AR)
    assert pad.shape == (n + 2 * c, n + 2 * c)
    for (i, j), v in ref.items():
        assert pad[i - 1 + c, j - 1 + c] == pytest.approx(v, abs=1e-12)
    assert len(ref) == (n + 2 * c) ** 2


def test_pad_wider_than_the_image_is_rejected():
    with pytest.raises(ValueError):
        blur.extension_matrix(4, 4, AR)


@pytest.mark.parametrize("p", [1, 3, 5, 9])
@pytest.mark.parametrize("method", ["direct", "fft"])
def test_affine_images_blur_in_closed_form(p, method):
    """The antireflective pad continues an affine image f = a + b y + e x
    exactly, so every output, the border ones included, is the valid
    convolution of the affine function:
    (A f)[i, j] = s f[i, j] + b sum H (c - a') + e sum H (c - b'), s = sum H."""
    n = 13
    g = synth.rng(p)
    H = rand_psf(g, p)
    c = (p - 1) // 2
    a0, b, e = 0.7, -0.3, 0.45
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    f = a0 + b * yy + e * xx
    s = H.sum()
    my = sum(H[ai, bi] * (c - ai) for ai in range(p) for bi in range(p))
    mx = sum(H[ai, bi] * (c - bi) for ai in range(p) for bi in range(p))
    want = s * f + b * my + e * mx
    fn = blur.blur_direct if method == "direct" else blur.blur_fft
    np.testing.assert_allclose(fn(f, H, AR), want, rtol=0, atol=1e-12)
    if p > 1:  # the reflective pad bends the affine image at the border
        assert np.abs(blur.blur_direct(f, H, blur.REFLECT) - want).max() > 1e-3


@pytest.mark.parametrize("bc", [blur.ZERO, blur.PERIODIC])
def test_reblur_is_the_transpose_for_zero_and_periodic(bc):
    """Section 2.2: imposing the boundary conditions on the rotated PSF gives
    A' = A^T for zero and periodic conditions."""
    n, p = 8, 5
    H = rand_psf(synth.rng(5 + bc), p)
    A = dense_of(lambda f: blur.blur_direct(f, H, bc), n)
    Ar = dense_of(lambda y: blur.reblur(y, H, bc, "direct"), n)
    np.testing.assert_allclose(Ar, A.T, rtol=0, atol=1e-13)


def test_blurT_uses_the_reblur_for_antireflective():
    n, p = 9, 5
    H = rand_psf(synth.rng(77), p)
    A = dense_of(lambda f: blur.blur_direct(f, H, AR), n)
    At = dense_of(lambda y: blur.blurT_direct(y, H, AR), n)
    Ar = dense_of(lambda y: blur.blurT(y, H, AR), n)
    np.testing.assert_allclose(At, A.T, rtol=0, atol=1e-13)  # the exact transpose stays available
    assert np.abs(Ar - A.T).max() > 1e-3                      # but the iterations use A'
    np.testing.assert_allclose(Ar, dense_of(lambda y: blur.blur_direct(y, H[::-1, ::-1], AR), n), atol=1e-13)
    np.testing.assert_allclose(dense_of(lambda y: blur.blurT(y, H, AR, "fft"), n), Ar, atol=1e-12)


@pytest.mark.parametrize("n,p", [(9, 3), (9, 5), (12, 7), (6, 5)])
def test_transform_diagonalises_the_antireflective_blur(n, p):
    """Dense Q (the antireflective blur of a quadrantally symmetric PSF, from
    the pinned pad) times the dense transform T x T equals T x T times the
    closed-form eigenvalues, column by column."""
    Hs = rand_psf(synth.rng(n * p), p, sym=True)
    Q = dense_of(lambda f: blur.blur_direct(f, Hs, AR), n)
    T2 = np.kron(precond.ar_basis(n), precond.ar_basis(n))
    lam = precond.ar_eigs(Hs, n)
    np.testing.assert_allclose(Q @ T2, T2 * lam.ravel()[None, :], rtol=0, atol=1e-13)


def test_linear_eigenvalue_is_the_psf_sum():
    """The linear basis functions are kept by the blur with eigenvalue sum H~
    (the symbol at frequency zero)."""
    Hs = rand_psf(synth.rng(3), 7, sym=True) * 1.7
    lam = precond.ar_eigs(Hs, 10)
    for k in (0, 9):
        for l in (0, 9):
            assert lam[k, l] == pytest.approx(Hs.sum(), rel=1e-14)


@pytest.mark.parametrize("n,p,alpha", [(9, 5, 0.3), (10, 3, 0.01), (7, 7, 1.0)])
def test_preconditioner_is_the_dense_inverse(n, p, alpha):
    """P r = (Q Q' + alpha I)^{-1} r with Q and Q' = the reblur of H~ built
    densely from the pinned blur (Algorithm 3 with antireflective conditions)."""
    g = synth.rng(n + p)
    H = rand_psf(g, p)
    Hs = precond.symmetrize(H)
    Q = dense_of(lambda f: blur.blur_direct(f, Hs, AR), n)
    Qr = dense_of(lambda y: blur.reblur(y, Hs, AR, "direct"), n)
    np.testing.assert_allclose(Qr, Q, atol=1e-14)   # H~ is invariant under the rotation
    r = g.standard_normal((n, n))
    want = np.linalg.solve(Q @ Qr + alpha * np.eye(n * n), r.ravel()).reshape(n, n)
    np.testing.assert_allclose(precond.apply(r, H, alpha, precond.AR), want, rtol=0, atol=1e-12)


def test_alg4_direction_is_dense():
    n, p, alpha = 9, 5, 0.05
    g = synth.rng(41)
    H = rand_psf(g, p)
    Q = dense_of(lambda f: blur.blur_direct(f, precond.symmetrize(H), AR), n)
    r = g.standard_normal((n, n))
    want = Q @ np.linalg.solve(Q @ Q + alpha * np.eye(n * n), r.ravel())
    np.testing.assert_allclose(alg4.apply_ct_prec(r, H, alpha, alg4.AR).ravel(), want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("pc", [precond.AR, precond.BCCB])
def test_opnorm_is_the_largest_eigenvalue_modulus(pc):
    n, p, alpha = 8, 5, 0.05
    H = rand_psf(synth.rng(8), p)
    A = dense_of(lambda f: blur.blur_direct(f, H, AR), n)
    Ar = dense_of(lambda y: blur.reblur(y, H, AR, "direct"), n)
    Pm = dense_of(lambda r: precond.apply(r, H, alpha, pc), n)
    want = np.abs(np.linalg.eigvals(Ar @ Pm @ A)).max()
    assert mlba.opnorm(H, n, AR, pc, alpha) == pytest.approx(want, rel=1e-6)  # a cluster at the top


@pytest.mark.parametrize("pc", [precond.AR, precond.NONE])
def test_threshold_free_run_is_preconditioned_landweber(pc):
    """mu = 0: with W^T W = I the synthesis u^k = W^T(delta z^k) obeys
    u^{k+1} = u^k + delta A' P (g - A u^k) (eq. MLBA2), written here with
    dense matrices of the pinned operators."""
    n, p, L, K, alpha, delta = 8, 5, 2, 6, 0.1, 0.7
    g0 = synth.rng(19)
    H = rand_psf(g0, p)
    gobs = g0.standard_normal((n, n))
    A = dense_of(lambda f: blur.blur_direct(f, H, AR), n)
    Ar = dense_of(lambda y: blur.reblur(y, H, AR, "direct"), n)
    Pm = dense_of(lambda r: precond.apply(r, H, alpha, pc), n)
    u = np.zeros(n * n)
    for _ in range(K):
        u = u + delta * Ar @ Pm @ (gobs.ravel() - A @ u)
    out = mlba.mlba(gobs, H, AR, pc, L, np.full(K, alpha), np.full(K + 1, delta), 0.0, K)
    np.testing.assert_allclose(out["f"].ravel(), u, rtol=0, atol=1e-11)


def test_opnorm_closed_form_for_a_symmetric_psf():
    """Symmetric PSF with the antireflective preconditioner: A = A' = Q, so
    A' P A = T Lambda^2 (Lambda^2 + alpha)^-1 T^-1 and its largest eigenvalue
    is the largest lambda^2 / (lambda^2 + alpha)."""
    n, p, alpha = 10, 5, 0.05
    H = synth.gaussian_psf(p, 1.2)
    lam = precond.ar_eigs(H, n)
    want = (lam * lam / (lam * lam + alpha)).max()
    assert mlba.opnorm(H, n, AR, precond.AR, alpha) == pytest.approx(want, rel=1e-6)
