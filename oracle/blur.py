"""Blur operator A and its transpose (oracle; test infrastructure only).

Paper, section 1 (eq. model2 / modeld): an n x n observation of an m x m
scene, m = n + p - 1, through a p x p PSF.  Section 2.1 (eq. Arect): the
rectangular n^2 x m^2 matrix A = M A_big keeps only the pixels of the field of
view, i.e. A f is the *valid* part of the 2-D convolution of f with H, and
A^T y is the *full* correlation of y with H.  Section 2.2 and Table 1: with an
imposed boundary condition the unknown is n x n and f is first extended by c =
(p-1)/2 pixels on every side (zero, periodic, mirrored or antireflected),
then blurred in valid mode.  The transpose of a boundary-condition blur is the
full correlation followed by the transpose of the extension (the pad
contributions folded back onto the pixels they were copied from).

Antireflective conditions (section 2.2): a pad pixel beyond an edge is twice
the edge pixel minus the pixel mirrored about it (the extension keeps the
normal derivative continuous); a corner pad pixel is antireflected in one
direction and then in the other.  The extension is therefore linear but not a
selection: row r of E holds 2 at the edge pixel and -1 at the mirrored one.
With these conditions the paper replaces A^T by the reblurring matrix A': the
same boundary conditions applied to the PSF rotated by 180 degrees.
:func:`blurT` (the operator the iterations use) returns A' for them, while
:func:`blurT_direct` and :func:`blurT_fft` stay the exact transposes.

Index convention: images are row-major arrays f[y, x]; H[a, b] with centre
(c, c).  With these conventions

    (A f)[i, j]   = sum_{a,b} H[a, b] fe[i + p-1-a, j + p-1-b],   0 <= i, j < n
    (A^T y)[k, l] = sum_{a,b} H[a, b] y[k-p+1+a, l-p+1+b]          (zero outside)

where fe = f for the rectangular model and fe = pad(f, c) otherwise.

Two implementations are kept: ``*_direct`` is the tap loop above (the
definition) and ``*_fft`` computes the same sums with scipy's FFT convolution,
the way the paper evaluates A (two FFTs of order m^2).  Tests cross-check them.
"""
from __future__ import annotations

import numpy as np
import scipy.signal
import scipy.sparse as sp

RECT, REFLECT, PERIODIC, ZERO, ANTIREFLECT = 0, 1, 2, 3, 4
BC_NAMES = {RECT: "rect", REFLECT: "reflect", PERIODIC: "periodic", ZERO: "zero",
            ANTIREFLECT: "antireflect"}


def unknown_side(n: int, p: int, bc: int) -> int:
    """Side of the unknown image: m = n + p - 1 for the rectangular model,
    n when a boundary condition is imposed (section 2)."""
    return n + p - 1 if bc == RECT else n


def extension_matrix(n: int, c: int, bc: int) -> sp.csr_matrix:
    """(n + 2c) x n matrix E with pad(f) = E f E^T along both axes.

    Row r (padded position r - c) selects the source pixel that Table 1 of the
    paper copies there: itself inside, its mirror image for reflective
    conditions (F_c, F_r: half-sample symmetric, position -1-i holds pixel i),
    its periodic image for periodic conditions, nothing for zero conditions.
    For antireflective conditions (section 2.2) position -i holds
    2 f[0] - f[i] and position n-1+i holds 2 f[n-1] - f[n-1-i] (1 <= i <= c,
    c <= n - 1); applying E along both axes antireflects the corners first in
    one direction and then in the other.
    """
    rows, cols, vals = [], [], []
    for r in range(n + 2 * c):
        x = r - c
        if bc == ANTIREFLECT:
            if 0 <= x < n:
                rows.append(r), cols.append(x), vals.append(1.0)
            else:
                edge = 0 if x < 0 else n - 1
                mirror = 2 * edge - x
                if not 0 <= mirror < n:
                    raise ValueError("antireflective pad wider than the image")
                rows += [r, r]
                cols += [edge, mirror]
                vals += [2.0, -1.0]
            continue
        if bc == PERIODIC:
            src = x % n
        elif bc == REFLECT:
            s = x % (2 * n)
            src = s if s < n else 2 * n - 1 - s
        elif bc == ZERO:
            if 0 <= x < n:
                src = x
            else:
                continue
        else:
            raise ValueError("extension only defined for boundary conditions")
        rows.append(r)
        cols.append(src)
        vals.append(1.0)
    return sp.csr_matrix((np.asarray(vals), (rows, cols)), shape=(n + 2 * c, n))


def _extend(f: np.ndarray, c: int, bc: int) -> np.ndarray:
    E = extension_matrix(f.shape[0], c, bc)
    return np.asarray(E @ (E @ f).T).T


def _fold(w: np.ndarray, n: int, c: int, bc: int) -> np.ndarray:
    """Transpose of _extend: E^T w E."""
    E = extension_matrix(n, c, bc)
    Et = E.T.tocsr()
    return np.asarray(Et @ (Et @ w).T).T


def blur_direct(f: np.ndarray, H: np.ndarray, bc: int) -> np.ndarray:
    """A f by the tap loop (section 2.1, eq. Arect; Table 1 for the padding)."""
    f = np.asarray(f, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    p = H.shape[0]
    c = (p - 1) // 2
    fe = f if bc == RECT else _extend(f, c, bc)
    n = fe.shape[0] - p + 1
    out = np.zeros((n, n))
    for a in range(p):
        for b in range(p):
            out += H[a, b] * fe[p - 1 - a:p - 1 - a + n, p - 1 - b:p - 1 - b + n]
    return out


def blurT_direct(y: np.ndarray, H: np.ndarray, bc: int) -> np.ndarray:
    """A^T y as the literal transpose of :func:`blur_direct`: every tap
    scatters y back onto the positions it read from, then the padding is
    folded (A^T = A_big^T M^T, section 2.1)."""
    y = np.asarray(y, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    p = H.shape[0]
    c = (p - 1) // 2
    n = y.shape[0]
    m = n + p - 1
    w = np.zeros((m, m))
    for a in range(p):
        for b in range(p):
            w[p - 1 - a:p - 1 - a + n, p - 1 - b:p - 1 - b + n] += H[a, b] * y
    if bc == RECT:
        return w
    return _fold(w, n, c, bc)


def blur_fft(f: np.ndarray, H: np.ndarray, bc: int) -> np.ndarray:
    """A f through FFT convolution (the paper's evaluation, section 2.1)."""
    f = np.asarray(f, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    c = (H.shape[0] - 1) // 2
    fe = f if bc == RECT else _extend(f, c, bc)
    return scipy.signal.fftconvolve(fe, H, mode="valid")


def blurT_fft(y: np.ndarray, H: np.ndarray, bc: int) -> np.ndarray:
    """A^T y through FFT correlation: full convolution with the PSF rotated by
    180 degrees, then the fold of the padding."""
    y = np.asarray(y, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    c = (H.shape[0] - 1) // 2
    w = scipy.signal.fftconvolve(y, H[::-1, ::-1], mode="full")
    if bc == RECT:
        return w
    return _fold(w, y.shape[0], c, bc)


def blur(f, H, bc, method: str = "auto"):
    if method == "direct" or (method == "auto" and f.shape[0] <= 96):
        return blur_direct(f, H, bc)
    return blur_fft(f, H, bc)


def reblur(y, H, bc, method: str = "auto"):
    """A' y (section 2.2): the blur of y under the same boundary conditions
    with the PSF rotated by 180 degrees."""
    return blur(np.asarray(y, dtype=np.float64), np.asarray(H, dtype=np.float64)[::-1, ::-1], bc, method)


def blurT(y, H, bc, method: str = "auto"):
    """The transpose the iterations use: A^T, or the reblurring A' for
    antireflective conditions (section 2.2)."""
    if bc == ANTIREFLECT:
        return reblur(y, H, bc, method)
    if method == "direct" or (method == "auto" and y.shape[0] <= 96):
        return blurT_direct(y, H, bc)
    return blurT_fft(y, H, bc)
