"""Algorithm 2 (section 4.2) — oracle; test infrastructure only.

The update direction of eq. (Alg2) is A^T t^n_{beta_n}, where t^n_{beta_n}
approximates (A A^T + alpha I)^{-1} r^n by beta_n steps of the conjugate
gradient method preconditioned by M = C C^T + alpha I (the spectral
preconditioner of Algorithm 1, or of Algorithm 3 for a DCT plan), started from
zero; equivalently the energy-norm minimiser of the symmetrised system
M^{-1/2} (A A^T + alpha I) M^{-1/2} y = M^{-1/2} r over the Krylov space of
size beta_n, t = M^{-1/2} y (eq. psys).  beta_n = min{beta_max, beta_tol}
(eq. bet): beta_tol is the first step count whose residual of that system,
relative to its right-hand side, is at most tol — in PCG terms
sqrt(res^T M^{-1} res / r^T M^{-1} r) <= tol (the paper: beta_max = 5,
tol = 1e-3).
"""
from __future__ import annotations

import numpy as np

from . import blur as _blur
from . import framelet as _fr
from . import precond as _pc
from .mlba import soft_threshold


def pcg_direction(r, H, bc, precond, alpha, beta_max=5, tol=1e-3):
    """t ~ (A A^T + alpha I)^{-1} r by preconditioned CG from t = 0; returns
    (t, steps taken)."""
    r = np.asarray(r, dtype=np.float64)

    def normal(v):
        return _blur.blur(_blur.blurT(v, H, bc), H, bc) + alpha * v

    def prec(v):
        return _pc.apply(v, H, alpha, precond)

    t = np.zeros_like(r)
    res = r.copy()
    zc = prec(res)
    d = zc.copy()
    rho = float(np.vdot(res, zc))
    rho0 = rho
    if rho0 == 0.0:
        return t, 0
    for j in range(1, beta_max + 1):
        q = normal(d)
        a = rho / float(np.vdot(d, q))
        t = t + a * d
        res = res - a * q
        zc = prec(res)
        rho_new = float(np.vdot(res, zc))
        if np.sqrt(rho_new / rho0) <= tol or j == beta_max:
            return t, j
        d = zc + (rho_new / rho) * d
        rho = rho_new
    return t, beta_max


def alg2(g, H, bc, precond, levels, alphas, deltas, mu, iters, beta_max=5, tol=1e-3, z0=None, k0=0) -> dict:
    """``iters`` steps of eq. (Alg2) from z0 (zero by default); alphas[k],
    deltas[k] indexed by the global step (deltas has one more entry for the
    returned image).  Returns dict(f, z, rnorm, betas)."""
    g = np.asarray(g, dtype=np.float64)
    n = g.shape[0]
    p = np.asarray(H).shape[0]
    N = _blur.unknown_side(n, p, bc)
    B = _fr.n_bands(levels)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (B,)).copy()
    z = np.zeros((B, N, N)) if z0 is None else np.array(z0, dtype=np.float64, copy=True)
    rnorm, betas = [], []
    for i in range(iters):
        k = k0 + i
        u = _fr.synthesis(deltas[k] * soft_threshold(z, mu), levels)
        r = g - _blur.blur(u, H, bc)
        rnorm.append(float(np.linalg.norm(r)))
        t, b = pcg_direction(r, H, bc, precond, float(alphas[k]), beta_max, tol)
        betas.append(b)
        z = z + _fr.analysis(_blur.blurT(t, H, bc), levels)
    f = _fr.synthesis(deltas[k0 + iters] * soft_threshold(z, mu), levels)
    return {"f": f, "z": z, "rnorm": np.asarray(rnorm), "betas": np.asarray(betas)}
