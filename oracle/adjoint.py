"""Reverse-mode gradient of K unrolled MLBA iterations (oracle; test
infrastructure only).

Forward (eq. MLBA2 of section 3 with the BCCB preconditioner of Algorithm 1,
rectangular blur of section 2.1, one step delta, per-band thresholds mu):

    z_0 = 0;  for k < K:  u_k = W^T(delta S_mu(z_k)),  r_k = g - A u_k,
                          t_k = P_alpha r_k,  z_{k+1} = z_k + W A^T t_k
    f = W^T(delta S_mu(z_K))

with A and P = (C C^T + alpha I)^{-1} both built from the PSF H.  Given
dl/df, the reverse sweep uses the almost-everywhere derivative of the soft
threshold (dS/dz = 1{|z| > mu}, dS/dmu = -sgn(z) 1{|z| > mu}, both 0 at
the kink |z| = mu) and, for the preconditioner, dP/dalpha = -P^2 and
d(CC^T) = F^* diag(d|Lambda|^2) F with |Lambda|^2 of the zero-padded PSF.
Everything is FP64; all forward states are kept (small problems only).
"""
from __future__ import annotations

import numpy as np

from . import blur as _blur
from . import framelet as _fr
from . import precond as _pc
from .mlba import soft_threshold


def psf_corr(x: np.ndarray, y: np.ndarray, p: int) -> np.ndarray:
    """d<y, A(H) x>/dH: entry (a, b) = sum_{i,j} y[i,j] x[i+p-1-a, j+p-1-b]
    (rectangular blur; x is m x m, y is n x n)."""
    n = y.shape[0]
    out = np.empty((p, p))
    for a in range(p):
        for b in range(p):
            out[a, b] = np.vdot(y, x[p - 1 - a:p - 1 - a + n, p - 1 - b:p - 1 - b + n])
    return out


def unrolled_forward(g, H, alpha, mu, delta, K, levels):
    g = np.asarray(g, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    n, p = g.shape[0], H.shape[0]
    N = n + p - 1
    B = _fr.n_bands(levels)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (B,)).copy()
    z = np.zeros((B, N, N))
    zs, us, ts = [z], [], []
    for _ in range(K):
        u = _fr.synthesis(delta * soft_threshold(z, mu), levels)
        r = g - _blur.blur(u, H, _blur.RECT)
        t = _pc.apply_bccb(r, H, alpha)
        z = z + _fr.analysis(_blur.blurT(t, H, _blur.RECT), levels)
        zs.append(z)
        us.append(u)
        ts.append(t)
    f = _fr.synthesis(delta * soft_threshold(z, mu), levels)
    return f, zs, us, ts


def unrolled_grad(g, H, alpha, mu, delta, K, levels, dl_df) -> dict:
    """Gradients of a loss with dl/df = dl_df w.r.t. mu (per band), alpha,
    the PSF H and the observation g."""
    g = np.asarray(g, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    n, p = g.shape[0], H.shape[0]
    B = _fr.n_bands(levels)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (B,)).copy()
    f, zs, us, ts = unrolled_forward(g, H, alpha, mu, delta, K, levels)
    big = np.zeros((n, n))
    big[:p, :p] = H
    lam = np.fft.fft2(big)

    def active(z):
        return (np.abs(z) > mu[:, None, None]).astype(np.float64)

    def band_sum(a):
        return a.reshape(B, -1).sum(axis=1)

    dmu = np.zeros(B)
    dalpha = 0.0
    dH = np.zeros((p, p))
    dg = np.zeros((n, n))
    xbar = _fr.analysis(np.asarray(dl_df, dtype=np.float64), levels)
    zK = zs[K]
    zbar = delta * active(zK) * xbar
    dmu += delta * band_sum(-np.sign(zK) * active(zK) * xbar)
    for k in range(K - 1, -1, -1):
        zk = zs[k]
        wbar = _fr.synthesis(zbar, levels)
        tbar = _blur.blur(wbar, H, _blur.RECT)
        rbar = _pc.apply_bccb(tbar, H, alpha)
        v = _fr.analysis(_blur.blurT(rbar, H, _blur.RECT), levels)
        dmu += delta * band_sum(np.sign(zk) * active(zk) * v)
        dalpha -= float(np.vdot(rbar, ts[k]))
        dg += rbar
        E = (np.conj(np.fft.fft2(rbar)) * np.fft.fft2(ts[k])).real / (n * n)
        spec = -2.0 * np.fft.fft2(E * np.conj(lam)).real[:p, :p]
        dH += psf_corr(wbar, ts[k], p) - psf_corr(us[k], rbar, p) + spec
        zbar = zbar - delta * active(zk) * v
    return {"f": f, "mu": dmu, "alpha": dalpha, "psf": dH, "g": dg}
