"""Algorithm 4 and Algorithm 4-NS (section 5) — oracle; test infrastructure only.

Algorithm 4 (eq. Alg4) solves the model equation L e = r with L = C W^T by
Tikhonov regularisation instead of using the normal equations: the update
direction is W C^T (C C^T + alpha I)^{-1} r, with C the square-boundary
approximation of the blur A:

  * BCCB: C is the blur under periodic boundary conditions (PSF centred at
    (c, c)), C = F^* diag(Lambda_c) F with Lambda_c the 2-D DFT of the PSF
    placed with its centre at the origin, so
    C^T (C C^T + alpha I)^{-1} r = F^{-1}[ conj(Lambda_c) F r / (|Lambda_c|^2 + alpha) ];
  * DCT: C is the reflective-boundary blur of the symmetrised PSF H~ (the
    matrix of Algorithm 3), symmetric and diagonalised by the orthonormal DCT-II:
    C^T (C C^T + alpha I)^{-1} r = C2^T[ lambda C2 r / (lambda^2 + alpha) ];
  * AR: C is the antireflective blur of H~ (sections 2.2 and 4.3), with C^T
    read as the reblurring C' = C (H~ is unchanged by the 180-degree rotation):
    C' (C C' + alpha I)^{-1} r = T[ lambda (T^-1 r) / (lambda^2 + alpha) ]
    with T the antireflective transform along both axes.

The method is only defined for square models (A imposes boundary conditions,
so A and C have the same size).

Algorithm 4-NS (eq. Alg4_revised) chooses alpha_n at every step from
alpha_n ||(C C^T + alpha_n I)^{-1} r^n|| = q_n ||r^n||,
q_n = max{q, 2 rho + (1 + rho) / tau_n}, tau_n = ||r^n|| / delta, and stops at
the first n with ||r^n|| <= tau delta, tau = (1 + 2 rho) / (1 - 2 rho)
(eq. Alg4_rev_12).  The root is unique (the left side increases with alpha from
below q_n ||r|| to ||r||); here it is found to machine precision by a bracketing
root finder on the spectral form of the norm (the paper's remark only asks for
"a few Newton steps").

Steps delta_n scale the thresholded coefficients as in the MLBA oracle
(x = delta S_mu(z)); the paper's choice is delta = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.optimize

from . import blur as _blur
from . import framelet as _fr
from . import precond as _pc
from .mlba import soft_threshold

BCCB, DCT, AR = _pc.BCCB, _pc.DCT, _pc.AR


def centred_eigs(H: np.ndarray, n: int) -> np.ndarray:
    """Lambda_c: eigenvalues of the periodic-boundary blur with the PSF centred
    at (c, c) (its kernel puts H[a, b] at ((a - c) mod n, (b - c) mod n))."""
    H = np.asarray(H, dtype=np.float64)
    p = H.shape[0]
    c = (p - 1) // 2
    big = np.zeros((n, n))
    big[:p, :p] = H
    return np.fft.fft2(np.roll(big, (-c, -c), axis=(0, 1)))


def apply_ct_prec(r: np.ndarray, H: np.ndarray, alpha: float, kind: int) -> np.ndarray:
    """C^T (C C^T + alpha I)^{-1} r (the direction of eq. Alg4 before W)."""
    r = np.asarray(r, dtype=np.float64)
    n = r.shape[0]
    if kind == BCCB:
        lam = centred_eigs(H, n)
        return np.fft.ifft2(np.conj(lam) * np.fft.fft2(r) / (np.abs(lam) ** 2 + alpha)).real
    if kind == DCT:
        lam = _pc.dct_eigs(_pc.symmetrize(H), n)
        c2 = scipy.fft.dctn(r, type=2, norm="ortho")
        return scipy.fft.idctn(lam * c2 / (lam * lam + alpha), type=2, norm="ortho")
    if kind == AR:
        lam = _pc.ar_eigs(_pc.symmetrize(H), n)
        return _pc.ar_filter(r, lam / (lam * lam + alpha))
    raise ValueError("Algorithm 4 needs the BCCB, DCT or antireflective preconditioner")


def tikhonov_norm(r: np.ndarray, H: np.ndarray, alpha: float, kind: int) -> float:
    """||(C C^T + alpha I)^{-1} r|| in closed spectral form."""
    return float(np.linalg.norm(_pc.apply(r, H, alpha, kind)))


def ns_alpha(r: np.ndarray, H: np.ndarray, q_n: float, kind: int) -> float:
    """The unique alpha > 0 with alpha ||(C C^T + alpha I)^{-1} r|| = q_n ||r||
    (eq. Alg4_rev_7), to machine precision.  Spectral form: with c_k the
    orthonormal transform coefficients of r and s_k the eigenvalues of C C^T,
    alpha^2 sum c_k^2 / (s_k + alpha)^2 = q_n^2 sum c_k^2."""
    r = np.asarray(r, dtype=np.float64)
    n = r.shape[0]
    if kind == BCCB:
        c2 = np.abs(np.fft.fft2(r)) ** 2 / (n * n)
        s = np.abs(centred_eigs(H, n)) ** 2
    elif kind == DCT:
        c2 = scipy.fft.dctn(r, type=2, norm="ortho") ** 2
        lam = _pc.dct_eigs(_pc.symmetrize(H), n)
        s = lam * lam
    else:
        raise ValueError("Algorithm 4-NS needs the BCCB or the DCT preconditioner")
    R = float(c2.sum())

    def phi(a):
        return a * a * float(np.sum(c2 / (s + a) ** 2)) - q_n * q_n * R

    hi = q_n * float(s.max()) / (1.0 - q_n) * 1.0001 + 1e-300
    while phi(hi) <= 0.0:
        hi *= 2.0
    return float(scipy.optimize.brentq(phi, 0.0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500))


def alg4(g, H, bc, precond, levels, alphas, deltas, mu, iters, z0=None, k0=0) -> dict:
    """``iters`` steps of eq. (Alg4) from z0 (zero by default); alphas[k],
    deltas[k] indexed by the global step (deltas has one more entry for the
    returned image)."""
    g = np.asarray(g, dtype=np.float64)
    if bc == _blur.RECT:
        raise ValueError("Algorithm 4 is defined for square (boundary-condition) models only")
    n = g.shape[0]
    B = _fr.n_bands(levels)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (B,)).copy()
    z = np.zeros((B, n, n)) if z0 is None else np.array(z0, dtype=np.float64, copy=True)
    rnorm = []
    for i in range(iters):
        k = k0 + i
        u = _fr.synthesis(deltas[k] * soft_threshold(z, mu), levels)
        r = g - _blur.blur(u, H, bc)
        rnorm.append(float(np.linalg.norm(r)))
        z = z + _fr.analysis(apply_ct_prec(r, H, float(alphas[k]), precond), levels)
    f = _fr.synthesis(deltas[k0 + iters] * soft_threshold(z, mu), levels)
    return {"f": f, "z": z, "rnorm": np.asarray(rnorm)}


def alg4_ns(g, H, bc, precond, levels, mu, noise: float, q: float = 0.5, rho: float = 1e-4,
            max_iters: int = 1000, delta: float = 1.0) -> dict:
    """Algorithm 4-NS from z = 0: returns the image W^T(delta S_mu(z^{n_delta}))
    at the first n with ||r^n|| <= tau * noise, the alpha_n used, the residual
    norms ||r^0 .. r^{n_delta}|| and n_delta (== max_iters if the stop never
    fired)."""
    g = np.asarray(g, dtype=np.float64)
    if bc == _blur.RECT:
        raise ValueError("Algorithm 4-NS is defined for square (boundary-condition) models only")
    if not (0.0 < rho < 0.5 and 2.0 * rho < q < 1.0 and noise > 0.0):
        raise ValueError("need 0 < rho < 1/2, 2 rho < q < 1 and a positive noise level")
    n = g.shape[0]
    B = _fr.n_bands(levels)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (B,)).copy()
    tau = (1.0 + 2.0 * rho) / (1.0 - 2.0 * rho)
    z = np.zeros((B, n, n))
    alphas, rnorm = [], []
    for it in range(max_iters + 1):
        u = _fr.synthesis(delta * soft_threshold(z, mu), levels)
        r = g - _blur.blur(u, H, bc)
        rn = float(np.linalg.norm(r))
        rnorm.append(rn)
        if rn <= tau * noise or it == max_iters:
            return {"f": u, "z": z, "alphas": np.asarray(alphas), "rnorm": np.asarray(rnorm), "iters": it}
        tau_n = rn / noise
        q_n = max(q, 2.0 * rho + (1.0 + rho) / tau_n)
        a = ns_alpha(r, H, q_n, precond)
        alphas.append(a)
        z = z + _fr.analysis(apply_ct_prec(r, H, a, precond), levels)
    raise AssertionError("unreachable")
