"""Spectral Tikhonov preconditioners (oracle; test infrastructure only).

Algorithm 1 (section 4.1, eq. Alg1): P = (C C^T + alpha I)^{-1} with C the
BCCB matrix of the PSF under periodic boundary conditions on the n x n residual
grid.  C = F^* diag(Lambda) F with Lambda the 2-D DFT of the zero-padded PSF,
so P r = F^{-1}[ F r / (|Lambda|^2 + alpha) ]; only |Lambda|^2 enters, so the
placement of the PSF inside the n x n array does not matter.

Algorithm 3 (section 4.3, eq. Alg3): the PSF is first made quadrantally
symmetric, H~(i,j) = (H(i,j) + H(-i,j) + H(i,-j) + H(-i,-j)) / 4 with offsets
taken from the PSF centre, and P = (Q Q^T + alpha I)^{-1} with Q the
reflective-boundary blur of H~, which the orthonormal 2-D DCT-II diagonalises
(section 4.1, the DCT alternative to the DFT).  Its eigenvalues are

    lambda[k, l] = sum_{a,b} H~[a, b] cos(pi k (a-c) / n) cos(pi l (b-c) / n)

(k the frequency along y, l along x), and P r = C2^T[ C2 r / (lambda^2 + alpha) ].

``NONE`` is P = I, which turns the iteration into the plain linearized
Bregman iteration (eq. iterLinBreg).

``AR`` is Algorithm 3 for antireflective boundary conditions (sections 2.2
and 4.3): Q is the antireflective blur of H~.  For a PSF symmetric about its
centre the antireflective extension of every vector of the basis

    t_0[k] = 1 - k/(n-1),   t_j[k] = sin(pi j k / (n-1)) (0 < j < n-1),
    t_{n-1}[k] = k/(n-1)

is the vector itself continued (the sines are odd about both ends, the linear
functions stay linear), so Q T = T Lambda with T = [t_0 .. t_{n-1}] along
each axis (the antireflective transform: the sine transform with the two
linear functions added) and

    lambda[k, l] = sum_{a,b} H~[a, b] cos(w_k (a-c)) cos(w_l (b-c)),
    w_j = pi j / (n-1) for the sines, w = 0 for the two linear functions.

Read with the paper's convention that Q^T stands for the reblurring Q' (the
antireflective blur of the rotated H~, i.e. Q itself), P = (Q Q' + alpha I)^-1
= T (Lambda^2 + alpha)^-1 T^-1.  T is not orthogonal; the oracle builds it
densely and applies T^-1 by solving with it.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg

BCCB, DCT, NONE, AR = 0, 1, 2, 3


def bccb_eigs_sq(H: np.ndarray, n: int) -> np.ndarray:
    """|Lambda|^2 on the n x n grid (Algorithm 1)."""
    H = np.asarray(H, dtype=np.float64)
    p = H.shape[0]
    big = np.zeros((n, n))
    big[:p, :p] = H
    lam = np.fft.fft2(big)
    return (lam * np.conj(lam)).real


def apply_bccb(r: np.ndarray, H: np.ndarray, alpha: float) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    s = bccb_eigs_sq(H, r.shape[0])
    return np.fft.ifft2(np.fft.fft2(r) / (s + alpha)).real


def symmetrize(H: np.ndarray) -> np.ndarray:
    """H~ of Algorithm 3: the average of H and its three reflections about the
    centre row and column."""
    H = np.asarray(H, dtype=np.float64)
    return (H + H[::-1, :] + H[:, ::-1] + H[::-1, ::-1]) / 4.0


def dct_eigs(Hs: np.ndarray, n: int) -> np.ndarray:
    """lambda[k, l] of the reflective-boundary blur of a quadrantally symmetric
    PSF (closed form above)."""
    Hs = np.asarray(Hs, dtype=np.float64)
    p = Hs.shape[0]
    c = (p - 1) // 2
    k = np.arange(n)[:, None]
    s = (np.arange(p) - c)[None, :]
    Cm = np.cos(np.pi * k * s / n)          # n x p
    return Cm @ Hs @ Cm.T


def apply_dct(r: np.ndarray, H: np.ndarray, alpha: float) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    lam = dct_eigs(symmetrize(H), r.shape[0])
    c2 = scipy.fft.dctn(r, type=2, norm="ortho")
    return scipy.fft.idctn(c2 / (lam * lam + alpha), type=2, norm="ortho")


def ar_basis(n: int) -> np.ndarray:
    """The n x n antireflective transform T (columns t_0 .. t_{n-1} above)."""
    N = n - 1
    k = np.arange(n, dtype=np.float64)
    T = np.empty((n, n))
    T[:, 0] = 1.0 - k / N
    T[:, n - 1] = k / N
    for j in range(1, n - 1):
        T[:, j] = np.sin(np.pi * j * k / N)
    return T


def ar_eigs(Hs: np.ndarray, n: int) -> np.ndarray:
    """lambda[k, l] of the antireflective blur of a quadrantally symmetric PSF
    (closed form above)."""
    Hs = np.asarray(Hs, dtype=np.float64)
    p = Hs.shape[0]
    c = (p - 1) // 2
    w = np.pi * np.arange(n, dtype=np.float64) / (n - 1)
    w[0] = w[n - 1] = 0.0
    Cm = np.cos(w[:, None] * (np.arange(p) - c)[None, :])   # n x p
    return Cm @ Hs @ Cm.T


def ar_filter(r: np.ndarray, lam_filter: np.ndarray) -> np.ndarray:
    """T (lam_filter * (T^-1 r T^-T)) T^T along both axes."""
    T = ar_basis(r.shape[0])
    lu = scipy.linalg.lu_factor(T)
    coef = scipy.linalg.lu_solve(lu, scipy.linalg.lu_solve(lu, r).T).T
    return T @ (coef * lam_filter) @ T.T


def apply_ar(r: np.ndarray, H: np.ndarray, alpha: float) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    lam = ar_eigs(symmetrize(H), r.shape[0])
    return ar_filter(r, 1.0 / (lam * lam + alpha))


def apply(r: np.ndarray, H: np.ndarray, alpha: float, kind: int) -> np.ndarray:
    if kind == AR:
        return apply_ar(r, H, alpha)
    if kind == BCCB:
        return apply_bccb(r, H, alpha)
    if kind == DCT:
        return apply_dct(r, H, alpha)
    if kind == NONE:
        return np.array(r, dtype=np.float64, copy=True)
    raise ValueError(f"unknown preconditioner {kind}")
