"""Pins of the oracle's reverse-mode gradient of unrolled MLBA: central finite
differences of the oracle's own forward pass (FP64, step small enough that no
coefficient crosses its threshold), and the definition of the PSF
correlation."""
import numpy as np
import pytest

import synth
from oracle import adjoint, blur


def _problem(seed, n=10, p=5, L=1):
    g = synth.rng(seed)
    H = g.random((p, p)) + 0.2
    H /= H.sum()
    truth = synth.shapes_image(n + p - 1, g, n_rect=4, n_disk=2)
    obs = synth.add_noise(blur.blur(truth, H, blur.RECT), synth.white_noise((n, n), g), 0.01)
    mu = g.uniform(0.002, 0.02, size=8 * L + 1)
    return obs, H, truth, mu


def _loss(obs, H, truth, alpha, mu, delta, K, L):
    f, *_ = adjoint.unrolled_forward(obs, H, alpha, mu, delta, K, L)
    return float(np.sum((f - truth) ** 2))


def _grad(obs, H, truth, alpha, mu, delta, K, L):
    f, *_ = adjoint.unrolled_forward(obs, H, alpha, mu, delta, K, L)
    return adjoint.unrolled_grad(obs, H, alpha, mu, delta, K, L, 2.0 * (f - truth))


def test_psf_corr_is_derivative_of_blur():
    g = synth.rng(1)
    n, p = 7, 3
    x = g.standard_normal((n + p - 1, n + p - 1))
    y = g.standard_normal((n, n))
    c = adjoint.psf_corr(x, y, p)
    for a in range(p):
        for b in range(p):
            E = np.zeros((p, p))
            E[a, b] = 1.0
            assert abs(c[a, b] - np.vdot(y, blur.blur_direct(x, E, blur.RECT))) < 1e-12


@pytest.mark.parametrize("L,K", [(1, 3), (2, 5)])
def test_gradient_matches_central_differences(L, K):
    obs, H, truth, mu = _problem(10 + L, L=L)
    alpha, delta = 0.1, 0.3
    gr = _grad(obs, H, truth, alpha, mu, delta, K, L)
    loss = lambda **kw: _loss(kw.get("obs", obs), kw.get("H", H), truth, kw.get("alpha", alpha),
                              kw.get("mu", mu), delta, K, L)
    # thresholds
    for b in range(len(mu)):
        h = 1e-7
        mp, mm = mu.copy(), mu.copy()
        mp[b] += h
        mm[b] -= h
        fd = (loss(mu=mp) - loss(mu=mm)) / (2 * h)
        assert abs(fd - gr["mu"][b]) <= 1e-5 * max(1.0, abs(fd)), (b, fd, gr["mu"][b])
    # alpha
    h = 1e-7
    fd = (loss(alpha=alpha + h) - loss(alpha=alpha - h)) / (2 * h)
    assert abs(fd - gr["alpha"]) <= 1e-5 * max(1.0, abs(fd))
    # every PSF entry (no renormalisation of the PSF inside the operator)
    p = H.shape[0]
    for a in range(p):
        for c in range(p):
            Hp, Hm = H.copy(), H.copy()
            Hp[a, c] += 1e-7
            Hm[a, c] -= 1e-7
            fd = (loss(H=Hp) - loss(H=Hm)) / 2e-7
            assert abs(fd - gr["psf"][a, c]) <= 1e-5 * max(1.0, abs(fd)), (a, c, fd, gr["psf"][a, c])
    # a few observation pixels
    for (i, j) in [(0, 0), (3, 7), (9, 9)]:
        op, om = obs.copy(), obs.copy()
        op[i, j] += 1e-7
        om[i, j] -= 1e-7
        fd = (loss(obs=op) - loss(obs=om)) / 2e-7
        assert abs(fd - gr["g"][i, j]) <= 1e-5 * max(1.0, abs(fd))


def test_directional_derivative_psf():
    obs, H, truth, mu = _problem(33, n=12, p=5, L=2)
    alpha, delta, K, L = 0.05, 0.25, 6, 2
    gr = _grad(obs, H, truth, alpha, mu, delta, K, L)
    V = synth.rng(7).standard_normal(H.shape)
    eps = 1e-7
    fd = (_loss(obs, H + eps * V, truth, alpha, mu, delta, K, L)
          - _loss(obs, H - eps * V, truth, alpha, mu, delta, K, L)) / (2 * eps)
    assert abs(fd - np.vdot(gr["psf"], V)) <= 1e-6 * max(1.0, abs(fd))
