"""Pins of the Algorithm 4 / 4-NS oracle (section 5) against dense linear
algebra, the blur oracle's boundary transposes, a closed form and its own
stopping rule."""
import numpy as np
import pytest

import synth
from oracle import alg4 as oa
from oracle import blur as ob
from oracle import framelet as ofr
from oracle import precond as opc


def _dense(H, n, bc):
    """The n^2 x n^2 matrix of the blur oracle (columns = blurred unit images)."""
    M = np.zeros((n * n, n * n))
    for j in range(n * n):
        e = np.zeros(n * n)
        e[j] = 1.0
        M[:, j] = ob.blur_direct(e.reshape(n, n), H, bc).ravel()
    return M


def _psf(p, seed, sym=False):
    g = synth.rng(seed)
    H = g.random((p, p)) + 0.1
    if sym:
        H = opc.symmetrize(H)
    return H / H.sum()


@pytest.mark.parametrize("n,p", [(8, 3), (8, 5), (12, 5)])
def test_centred_eigs_diagonalise_periodic_blur(n, p):
    H = _psf(p, n + p)
    v = synth.rng(1).standard_normal((n, n))
    lam = oa.centred_eigs(H, n)
    assert np.allclose(np.fft.ifft2(lam * np.fft.fft2(v)).real, ob.blur_direct(v, H, ob.PERIODIC), atol=1e-13)
    # |Lambda_c|^2 is the spectrum of Algorithm 1 (placement does not matter there)
    assert np.allclose(np.abs(lam) ** 2, opc.bccb_eigs_sq(H, n), atol=1e-13)


@pytest.mark.parametrize("n,p,alpha", [(8, 3, 0.05), (8, 5, 0.2), (12, 5, 0.01)])
def test_bccb_direction_dense_and_transpose(n, p, alpha):
    H = _psf(p, 3 * n + p)  # not symmetric: the phase of Lambda_c matters
    r = synth.rng(2).standard_normal((n, n))
    got = oa.apply_ct_prec(r, H, alpha, oa.BCCB)
    C = _dense(H, n, ob.PERIODIC)
    ref = C.T @ np.linalg.solve(C @ C.T + alpha * np.eye(n * n), r.ravel())
    assert np.allclose(got.ravel(), ref, atol=1e-12)
    # = A^T P r for the periodic model, through the blur oracle's own transpose
    assert np.allclose(got, ob.blurT_direct(opc.apply_bccb(r, H, alpha), H, ob.PERIODIC), atol=1e-12)


@pytest.mark.parametrize("n,p,alpha", [(8, 3, 0.05), (8, 5, 0.3), (10, 5, 0.02)])
def test_dct_direction_dense(n, p, alpha):
    H = _psf(p, 5 * n + p)
    Hs = opc.symmetrize(H)
    r = synth.rng(3).standard_normal((n, n))
    got = oa.apply_ct_prec(r, H, alpha, oa.DCT)
    Q = _dense(Hs, n, ob.REFLECT)
    assert np.allclose(Q, Q.T, atol=1e-14)
    ref = Q.T @ np.linalg.solve(Q @ Q.T + alpha * np.eye(n * n), r.ravel())
    assert np.allclose(got.ravel(), ref, atol=1e-12)


@pytest.mark.parametrize("L", [1, 2])
def test_periodic_closed_form(L):
    """Periodic model, BCCB, mu = 0, unit step: W^T W = I makes f^{n+1} =
    f^n + C^T (C C^T + alpha_n)^{-1} (g - C f^n), i.e.
    F f^K = (1 - prod_n alpha_n / (|Lambda|^2 + alpha_n)) F g / Lambda."""
    n, p = 16, 5
    H = _psf(p, 77)
    g = synth.rng(4).standard_normal((n, n))
    alphas = np.array([0.3, 0.1, 0.05, 0.2, 0.02, 0.08])
    K = len(alphas)
    res = oa.alg4(g, H, ob.PERIODIC, oa.BCCB, L, alphas, np.ones(K + 1), 0.0, K)
    lam = oa.centred_eigs(H, n)
    s = np.abs(lam) ** 2
    prod = np.prod([a / (s + a) for a in alphas], axis=0)
    ref = np.fft.ifft2((1.0 - prod) * np.fft.fft2(g) / lam).real
    assert np.allclose(res["f"], ref, atol=1e-10)


@pytest.mark.parametrize("kind,bc", [(oa.BCCB, ob.ZERO), (oa.BCCB, ob.PERIODIC), (oa.DCT, ob.REFLECT)])
@pytest.mark.parametrize("q", [0.5, 0.9])
def test_ns_alpha_solves_its_equation(kind, bc, q):
    n, p = 8, 5
    H = _psf(p, 11, sym=(kind == oa.DCT))
    r = synth.rng(5).standard_normal((n, n))
    a = oa.ns_alpha(r, H, q, kind)
    C = _dense(H, n, ob.PERIODIC) if kind == oa.BCCB else _dense(opc.symmetrize(H), n, ob.REFLECT)
    y = np.linalg.solve(C @ C.T + a * np.eye(n * n), r.ravel())
    assert abs(a * np.linalg.norm(y) - q * np.linalg.norm(r)) <= 1e-11 * np.linalg.norm(r)
    # and it is the only root: the left side increases with alpha
    ys = [np.linalg.norm(np.linalg.solve(C @ C.T + b * np.eye(n * n), r.ravel())) * b for b in (0.5 * a, 2.0 * a)]
    assert ys[0] < q * np.linalg.norm(r) < ys[1]


@pytest.mark.parametrize("kind,bc", [(oa.BCCB, ob.ZERO), (oa.DCT, ob.REFLECT)])
def test_ns_stops_by_the_discrepancy_rule_and_replays(kind, bc):
    """The iteration stops at the first n with ||r^n|| <= tau delta; replaying
    Algorithm 4 with the alpha_n it chose reproduces it."""
    n, p, L = 24, 5, 1
    gen = synth.rng(12)
    H = synth.gaussian_psf(p, 1.0)
    truth = synth.shapes_image(n, gen, n_rect=4, n_disk=2)
    b = ob.blur(truth, H, bc)
    g = synth.add_noise(b, synth.white_noise((n, n), gen), 0.01)
    noise = synth.noise_norm(b, 0.01)
    rho = 1e-4
    res = oa.alg4_ns(g, H, bc, kind, L, 2e-3, noise, q=0.5, rho=rho, max_iters=200)
    tau = (1 + 2 * rho) / (1 - 2 * rho)
    k = res["iters"]
    assert 0 < k < 200
    assert res["rnorm"][k] <= tau * noise < res["rnorm"][:k].min()
    rep = oa.alg4(g, H, bc, kind, L, res["alphas"], np.ones(k + 1), 2e-3, k)
    assert np.allclose(rep["f"], res["f"], atol=1e-12)
    assert np.allclose(rep["rnorm"], res["rnorm"][:k], rtol=1e-12)


def test_alg4_rejects_rectangular_model():
    with pytest.raises(ValueError):
        oa.alg4(np.zeros((8, 8)), _psf(3, 1), ob.RECT, oa.BCCB, 1, [0.1], [1.0, 1.0], 0.0, 1)
