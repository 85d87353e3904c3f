"""Undecimated linear B-spline tight framelet (oracle; test infrastructure only).

Paper, section 6.1: the masks

    b0 = 1/4 [1, 2, 1],   b1 = sqrt(2)/4 [1, 0, -1],   b2 = 1/4 [-1, 2, -1]

define N x N one-dimensional filters B0, B1, B2 under reflective boundary
conditions; the 2-D filters are the tensor products B_{i,j} = B_i (x) B_j and
the analysis operator stacks them, W = [B_00; B_01; ...; B_22].  Section 3 and
eq. (wavecoeff): the synthesis operator is the transpose W^T and W^T W = I.

Readings (the paper is silent or inconsistent on these):
  * the printed matrices of section 6.1 swap the labels of B1 and B2 and the
    printed B2 lacks the sqrt(2) of its mask; the masks are authoritative.
    With the printed rows, (B1-mask v)[x] = sqrt(2)/4 (v[x+d] - v[x-d]).
  * several levels (the paper uses the multilevel decomposition of its [COS]
    reference): undecimated a-trous, level l uses dilation d = 2^(l-1) and
    is applied to the low-pass output of level l-1, with the same reflective
    extension at every level and no per-level normalisation.
  * reflective extension: position x outside [0, N) takes pixel
    ext(x) = s if s < N else 2N-1-s, with s = x mod 2N (half-sample symmetric,
    matching the first row 1/4 [3 1] of the printed B0).
  * band (i, j) applies B_i along x (columns) and B_j along y (rows): for the
    paper's column stacking, (B_i (x) B_j) vec(F) = vec(B_j F B_i^T).
  * band order of a level: (0,1),(0,2),(1,0),(1,1),(1,2),(2,0),(2,1),(2,2);
    the coefficient vector is [v_L, level-1 bands, ..., level-L bands] where
    v_L is the final low-pass image (band 0).  For one level this is the
    paper's [B_00; B_01; ...; B_22] with B_00 moved first.

Synthesis is not written separately: it is the sparse transpose of the very
matrices used by the analysis, so W^T is W's adjoint by construction.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

MASKS = (
    (0.25, 0.5, 0.25),                              # b0 at offsets -d, 0, +d
    (-math.sqrt(2) / 4, 0.0, math.sqrt(2) / 4),     # b1
    (-0.25, 0.5, -0.25),                            # b2
)
PAIRS = ((0, 1), (0, 2), (1, 0), (1, 1), (1, 2), (2, 0), (2, 1), (2, 2))


def n_bands(levels: int) -> int:
    return 8 * levels + 1


def band_index(level: int, q: int) -> int:
    """Position of pair PAIRS[q] of ``level`` (1-based) in the coefficient stack."""
    return 1 + 8 * (level - 1) + q


def ext(x: int, N: int) -> int:
    s = x % (2 * N)
    return s if s < N else 2 * N - 1 - s


def filter_matrix(i: int, N: int, d: int) -> sp.csr_matrix:
    """N x N matrix of mask b_i with dilation d under reflective extension:
    (B v)[x] = sum_k b_i[k] v[ext(x + k d)], k in {-1, 0, 1}."""
    rows, cols, vals = [], [], []
    for x in range(N):
        for k, coef in zip((-1, 0, 1), MASKS[i]):
            if coef == 0.0:
                continue
            rows.append(x)
            cols.append(ext(x + k * d, N))
            vals.append(coef)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))  # duplicates are summed


def _along_y(M, v):
    return np.asarray(M @ v)


def _along_x(M, v):
    return np.asarray(M @ v.T).T


def analysis(f: np.ndarray, levels: int) -> np.ndarray:
    """z = W f, shape (8*levels + 1, N, N)."""
    f = np.asarray(f, dtype=np.float64)
    N = f.shape[0]
    out = np.empty((n_bands(levels), N, N))
    v = f
    for lev in range(1, levels + 1):
        d = 2 ** (lev - 1)
        M = [filter_matrix(i, N, d) for i in range(3)]
        hx = [_along_x(M[i], v) for i in range(3)]        # B_i along x
        for q, (i, j) in enumerate(PAIRS):
            out[band_index(lev, q)] = _along_y(M[j], hx[i])
        v = _along_y(M[0], hx[0])
    out[0] = v
    return out


def synthesis(z: np.ndarray, levels: int) -> np.ndarray:
    """f = W^T z: the transpose of :func:`analysis`, level L down to 1."""
    z = np.asarray(z, dtype=np.float64)
    N = z.shape[-1]
    v = z[0]
    for lev in range(levels, 0, -1):
        d = 2 ** (lev - 1)
        Mt = [filter_matrix(i, N, d).T.tocsr() for i in range(3)]
        # sum over (i, j) of B_i^T along x of (B_j^T along y of band(i, j))
        acc_y = [None, None, None]
        acc_y[0] = _along_y(Mt[0], v)
        for q, (i, j) in enumerate(PAIRS):
            t = _along_y(Mt[j], z[band_index(lev, q)])
            acc_y[i] = t if acc_y[i] is None else acc_y[i] + t
        v = sum(_along_x(Mt[i], acc_y[i]) for i in range(3))
    return v


def dense_1d(i: int, N: int, d: int = 1) -> np.ndarray:
    return filter_matrix(i, N, d).toarray()
