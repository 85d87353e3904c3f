"""The modified linearized Bregman iteration (oracle; test infrastructure only).

Paper, section 3:
  * eq. (soft): S_mu(x) = sgn(x) max(|x| - mu, 0), componentwise;
  * eq. (MLBA):  z^{k+1} = z^k + K^T P (g - K x^k),  x^{k+1} = lambda S_mu(z^{k+1}),
    z^0 = x^0 = 0, with K = A W^T (eq. K);
  * eq. (MLBA2): the synthesis form actually run, z^{k+1} = z^k + W A^T P (g -
    A W^T x^k), with the preconditioner of eq. (Pstandard) or Algorithms 1/3.
  * Theorem (convergence of MLBA): converges when 0 < lambda < 1/||K^T P K||;
    since W^T W = I, ||K^T P K|| = ||A^T P A||.

Readings (recorded with the other readings of the paper):
  * the scale lambda of eq. (MLBA) is the step called ``delta`` here, applied
    as x^k = delta_k S_mu(z^k); a nonpositive request selects
    delta_k = 0.9 / max(||A^T P_{alpha_k} A||, 0.9), which keeps the
    convergence condition with a 10 % margin (the paper sets lambda = 1, which
    is only safe when alpha is large enough, section 4.1);
  * mu may be one value or one value per band (band 0 is the low-pass);
  * the geometric schedule alpha_k = max(alpha_0 r^k, alpha_floor) is not
    the paper's; iteration k uses alpha_k and delta_k, and the returned image
    is W^T (delta_K S_mu(z^K));
  * with antireflective boundary conditions A^T stands for the reblurring
    matrix A' throughout (section 2.2), so the update is W A' P r and the
    norm of the step rule is the largest eigenvalue modulus of A' P A.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import blur as _blur
from . import framelet as _fr
from . import precond as _pc


def soft_threshold(x: np.ndarray, mu) -> np.ndarray:
    """S_mu of eq. (soft); ``mu`` broadcasts over leading (band) axes."""
    x = np.asarray(x, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    if mu.ndim == 1 and x.ndim == 3:
        mu = mu[:, None, None]
    return np.sign(x) * np.maximum(np.abs(x) - mu, 0.0)


def alpha_table(kind: int, alpha0: float, count: int, ratio: float = 1.0,
                floor: float = 0.0) -> np.ndarray:
    """alpha_k for k = 0 .. count-1: constant (kind 0) or geometric (kind 1)."""
    k = np.arange(count, dtype=np.float64)
    if kind == 0:
        return np.full(count, float(alpha0))
    return np.maximum(alpha0 * ratio ** k, floor)


def opnorm(H: np.ndarray, n: int, bc: int, precond: int, alpha: float,
           tol: float = 1e-10) -> float:
    """||A^T P_alpha A|| (largest eigenvalue of the symmetric positive
    semidefinite operator) by Lanczos; for antireflective conditions the
    largest eigenvalue modulus of A' P_alpha A by Arnoldi."""
    p = H.shape[0]
    N = _blur.unknown_side(n, p, bc)

    def mv(v):
        f = v.reshape(N, N)
        r = _blur.blur(f, H, bc)
        t = _pc.apply(r, H, alpha, precond)
        return _blur.blurT(t, H, bc).ravel()

    op = spla.LinearOperator((N * N, N * N), matvec=mv, dtype=np.float64)
    v0 = np.random.Generator(np.random.PCG64(12345)).standard_normal(N * N)
    if bc == _blur.ANTIREFLECT:
        # A' P A is not symmetric (section 2.2's reblurring): the largest
        # eigenvalue modulus by Arnoldi instead of Lanczos
        val = spla.eigs(op, k=1, which="LM", v0=v0, tol=tol, return_eigenvectors=False)
        return float(abs(val[0]))
    val = spla.eigsh(op, k=1, which="LA", v0=v0, tol=tol, return_eigenvectors=False)
    return float(val[0])


def delta_auto(norm_value: float) -> float:
    return 0.9 / max(norm_value, 0.9)


def delta_table(H, n, bc, precond, alphas, delta: float, count: int) -> np.ndarray:
    """delta_k for k = 0 .. count-1 (``alphas`` holds at least one entry; the
    last alpha is reused past its end).  The automatic step uses the norm to
    opnorm's default tolerance (converged to rounding)."""
    if delta > 0:
        return np.full(count, float(delta))
    cache = {}
    out = np.empty(count)
    for k in range(count):
        a = float(alphas[min(k, len(alphas) - 1)])
        if a not in cache:
            cache[a] = delta_auto(opnorm(H, n, bc, precond, a))
        out[k] = cache[a]
    return out


def mlba(g: np.ndarray, H: np.ndarray, bc: int, precond: int, levels: int,
         alphas, deltas, mu, iters: int, z0: np.ndarray | None = None,
         k0: int = 0, method: str = "auto") -> dict:
    """Run ``iters`` iterations of eq. (MLBA2) from z0 (zero by default).

    alphas[k], deltas[k] are indexed by the global iteration number k0 + i;
    ``deltas`` needs one more entry for the returned image.
    Returns dict(f=W^T(delta S_mu(z)), z=z, rnorm=[||g - A u^k||]).
    """
    g = np.asarray(g, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    n = g.shape[0]
    p = H.shape[0]
    N = _blur.unknown_side(n, p, bc)
    B = _fr.n_bands(levels)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (B,)).copy()
    z = np.zeros((B, N, N)) if z0 is None else np.array(z0, dtype=np.float64, copy=True)
    rnorm = []
    for i in range(iters):
        k = k0 + i
        x = deltas[k] * soft_threshold(z, mu)
        u = _fr.synthesis(x, levels)
        r = g - _blur.blur(u, H, bc, method)
        rnorm.append(float(np.linalg.norm(r)))
        t = _pc.apply(r, H, float(alphas[k]), precond)
        w = _blur.blurT(t, H, bc, method)
        z = z + _fr.analysis(w, levels)
    f = _fr.synthesis(deltas[k0 + iters] * soft_threshold(z, mu), levels)
    return {"f": f, "z": z, "rnorm": np.asarray(rnorm)}
