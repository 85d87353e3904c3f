"""Seeded synthetic workloads for frame-based deblurring.

This module produces the raw ingredients of a test problem and nothing else:
true images, point spread functions, white-noise directions and the scalar
parameters of each workload.  It contains none of the restoration method's
arithmetic (no blur, no transform, no framelet, no threshold): the observed
image ``g = A f + eta`` is formed by whoever owns a blur operator, and
:func:`add_noise` only rescales a given noise direction to the requested level.

The shapes follow the paper's experiments (section 6: 256x256 scenes, 1-2 %
white Gaussian noise, PSFs up to 31x31, Gaussian / motion / out-of-focus
blurs); the sizes and parameters are those of the workloads listed in
:data:`WORKLOADS`.  Every array is float64; every draw comes from a PCG64
generator seeded explicitly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng",
    "shapes_image",
    "gaussian_psf",
    "motion_psf",
    "disk_psf",
    "white_noise",
    "add_noise",
    "Workload",
    "WORKLOADS",
    "make_workload",
    "batched_workloads",
]

# boundary / preconditioner codes (plain integers so both sides can use them)
RECT, REFLECT, PERIODIC, ZERO, ANTIREFLECT = 0, 1, 2, 3, 4
BCCB, DCT, NONE, AR = 0, 1, 2, 3


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for ``seed``."""
    return np.random.Generator(np.random.PCG64(int(seed)))


# ---------------------------------------------------------------------------
# true images
# ---------------------------------------------------------------------------

def shapes_image(m: int, g: np.random.Generator, n_rect: int = 12, n_disk: int = 6,
                 n_bumps: int = 0, texture: float = 0.0) -> np.ndarray:
    """An m x m scene of painted rectangles and disks, optional smooth Gaussian
    bumps and an optional band-limited texture, min-max normalised to [0, 1].

    rectangles: sides ~ U[m/16, m/3], values ~ U[0, 1], painted in order;
    disks: radius ~ U[m/32, m/8]; bumps: sigma ~ U[m/40, m/8], amplitude
    ~ U[0, 1], added; texture: a sum of 32 plane waves with frequencies below
    0.1 cycle/pixel and random phases, scaled to peak amplitude ``texture``.
    """
    img = np.zeros((m, m))
    yy, xx = np.mgrid[0:m, 0:m].astype(np.float64)
    for _ in range(n_rect):
        h = g.uniform(m / 16, m / 3)
        w = g.uniform(m / 16, m / 3)
        y0 = g.uniform(-h / 2, m - h / 2)
        x0 = g.uniform(-w / 2, m - w / 2)
        val = g.uniform(0.0, 1.0)
        mask = (yy >= y0) & (yy < y0 + h) & (xx >= x0) & (xx < x0 + w)
        img[mask] = val
    for _ in range(n_disk):
        r = g.uniform(m / 32, m / 8)
        cy, cx = g.uniform(0, m), g.uniform(0, m)
        val = g.uniform(0.0, 1.0)
        img[(yy - cy) ** 2 + (xx - cx) ** 2 <= r * r] = val
    for _ in range(n_bumps):
        s = g.uniform(m / 40, m / 8)
        cy, cx = g.uniform(0, m), g.uniform(0, m)
        a = g.uniform(0.0, 1.0)
        img += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
    if texture > 0:
        tex = np.zeros((m, m))
        for _ in range(32):
            f = g.uniform(0.0, 0.1)
            th = g.uniform(0.0, math.pi)
            ph = g.uniform(0.0, 2 * math.pi)
            tex += np.cos(2 * math.pi * f * (math.cos(th) * xx + math.sin(th) * yy) + ph)
        tex *= texture / max(np.abs(tex).max(), 1e-300)
        img += tex
    lo, hi = img.min(), img.max()
    if hi > lo:
        img = (img - lo) / (hi - lo)
    return img


# ---------------------------------------------------------------------------
# point spread functions (p x p, nonnegative, sum 1, centred at (c, c))
# ---------------------------------------------------------------------------

def _centred_grid(p: int):
    c = (p - 1) / 2.0
    y, x = np.mgrid[0:p, 0:p].astype(np.float64)
    return y - c, x - c


def gaussian_psf(p: int, sigma: float) -> np.ndarray:
    y, x = _centred_grid(p)
    h = np.exp(-(x * x + y * y) / (2.0 * sigma * sigma))
    return h / h.sum()


def motion_psf(p: int, length: float, theta: float, samples: int = 4001) -> np.ndarray:
    """A straight motion streak of the given length through the centre at angle
    ``theta``, rasterised by bilinear splatting of ``samples`` points."""
    c = (p - 1) / 2.0
    h = np.zeros((p, p))
    t = np.linspace(-length / 2.0, length / 2.0, samples)
    xs = c + t * math.cos(theta)
    ys = c + t * math.sin(theta)
    x0 = np.floor(xs).astype(int)
    y0 = np.floor(ys).astype(int)
    fx = xs - x0
    fy = ys - y0
    for dy, dx, wgt in ((0, 0, (1 - fy) * (1 - fx)), (0, 1, (1 - fy) * fx),
                        (1, 0, fy * (1 - fx)), (1, 1, fy * fx)):
        yi, xi = y0 + dy, x0 + dx
        ok = (yi >= 0) & (yi < p) & (xi >= 0) & (xi < p)
        np.add.at(h, (yi[ok], xi[ok]), wgt[ok])
    return h / h.sum()


def disk_psf(p: int, radius: float) -> np.ndarray:
    y, x = _centred_grid(p)
    h = (x * x + y * y <= radius * radius).astype(np.float64)
    return h / h.sum()


# ---------------------------------------------------------------------------
# noise
# ---------------------------------------------------------------------------

def white_noise(shape, g: np.random.Generator) -> np.ndarray:
    """A standard normal direction xi (unscaled)."""
    return g.standard_normal(shape)


def add_noise(blurred: np.ndarray, xi: np.ndarray, level: float) -> np.ndarray:
    """``blurred + eta`` with ``eta = level * ||blurred|| * xi / ||xi||`` so the
    noise norm is exactly ``level * ||blurred||``."""
    blurred = np.asarray(blurred, dtype=np.float64)
    scale = level * np.linalg.norm(blurred) / np.linalg.norm(xi)
    return blurred + scale * xi


def noise_norm(blurred: np.ndarray, level: float) -> float:
    return float(level * np.linalg.norm(np.asarray(blurred, dtype=np.float64)))


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    """One restoration problem: truth (m x m), PSF (p x p), noise direction
    (n x n) plus the method's parameters.  ``g`` is left for the caller."""
    name: str
    n: int
    p: int
    truth: np.ndarray
    psf: np.ndarray
    xi: np.ndarray
    noise_level: float
    bc: int = RECT
    precond: int = BCCB
    levels: int = 1
    alpha0: float = 0.05
    alpha_kind: int = 0          # 0 constant, 1 geometric
    alpha_ratio: float = 1.0
    alpha_floor: float = 0.0
    mu: float = 1e-3
    delta: float = 1.0           # <= 0: automatic step 0.9 / max(||A^T P A||, 0.9)
    iters: int = 50
    extra: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.n + self.p - 1

    @property
    def N(self) -> int:
        return self.m if self.bc == RECT else self.n

    @property
    def bands(self) -> int:
        return 8 * self.levels + 1


def _cfg1(seed=1):
    g = rng(seed)
    n, p = 64, 9
    truth = shapes_image(n + p - 1, g, n_rect=12, n_disk=6)
    psf = gaussian_psf(p, 2.0)
    xi = white_noise((n, n), g)
    return Workload("plain-fp64-72", n, p, truth, psf, xi, 0.01, RECT, BCCB, 1,
                    alpha0=0.05, mu=1e-3, delta=1.0, iters=50)


def _cfg2(variant: int, seed=2):
    g = rng(seed)
    n, p = 512, 17
    truth = shapes_image(n + p - 1, g, n_rect=8, n_disk=4, n_bumps=20)
    theta = g.uniform(0.0, math.pi)
    psf = motion_psf(p, 15.0, theta)
    xi = white_noise((n, n), g)
    if variant == 1:
        return Workload("rect-bccb-512", n, p, truth, psf, xi, 0.01, RECT, BCCB, 2,
                        alpha0=0.05, mu=1e-3, delta=0.0, iters=200, extra={"theta": theta})
    if variant == 2:
        return Workload("reflect-dct-512", n, p, truth, psf, xi, 0.01, REFLECT, DCT, 2,
                        alpha0=0.05, mu=1e-3, delta=0.0, iters=200, extra={"theta": theta})
    return Workload("rect-bccb-geometric-512", n, p, truth, psf, xi, 0.01, RECT, BCCB, 2,
                    alpha0=0.5, alpha_kind=1, alpha_ratio=0.8, alpha_floor=0.02,
                    mu=1e-3, delta=0.0, iters=200, extra={"theta": theta})


def _cfg3(seed=3):
    g = rng(seed)
    n, p = 2048, 31
    truth = shapes_image(n + p - 1, g, n_rect=28, n_disk=12, texture=0.2)
    psf = disk_psf(p, 15.0)
    xi = white_noise((n, n), g)
    return Workload("rect-bccb-2048", n, p, truth, psf, xi, 0.005, RECT, BCCB, 3,
                    alpha0=0.02, mu=1e-3, delta=0.0, iters=300)


def _cfg5(seed=5, count=16):
    out = []
    for i in range(count):
        g = rng(seed * 1000 + i)
        n, p = 256, 15
        truth = shapes_image(n + p - 1, g, n_rect=10, n_disk=5, n_bumps=6)
        psf = gaussian_psf(p, 2.5)
        xi = white_noise((n, n), g)
        out.append(Workload(f"unrolled-256-{i}", n, p, truth, psf, xi, 0.01, RECT, BCCB, 2,
                            alpha0=0.05, mu=1e-3, delta=0.0, iters=30,
                            extra={"ckpt_every": 5}))
    return out


def batched_workloads(seed: int = 4, count: int = 64, sides=(128, 192, 256, 384, 512, 768, 1024),
                      iters: int = 100):
    """The uneven batch: sides drawn from ``sides``, Gaussian PSFs with
    sigma ~ U[1, 4] and odd size in [9, 25], noise ~ U[0.5 %, 2 %],
    alpha ~ U[0.01, 0.2], 2-level framelet."""
    g = rng(seed)
    out = []
    for i in range(count):
        n = int(g.choice(np.asarray(sides)))
        p = int(g.choice(np.arange(9, 26, 2)))
        sigma = float(g.uniform(1.0, 4.0))
        level = float(g.uniform(0.005, 0.02))
        alpha = float(g.uniform(0.01, 0.2))
        gi = rng(seed * 100000 + i)
        truth = shapes_image(n + p - 1, gi, n_rect=10, n_disk=5, n_bumps=4)
        psf = gaussian_psf(p, sigma)
        xi = white_noise((n, n), gi)
        out.append(Workload(f"batch-{i}-{n}", n, p, truth, psf, xi, level, RECT, BCCB, 2,
                            alpha0=alpha, mu=1e-3, delta=0.0, iters=iters,
                            extra={"sigma": sigma}))
    return out


def _cfg_ar(seed=6):
    """Antireflective model with the antireflective-transform preconditioner
    (Alg-BC3 of Example 4): 31 x 31 Gaussian PSF of standard deviation 2.5,
    2 % noise, the observation the valid part of a larger scene."""
    g = rng(seed)
    n, p = 1025, 31
    truth = shapes_image(n + p - 1, g, n_rect=20, n_disk=10, n_bumps=10, texture=0.2)
    psf = gaussian_psf(p, 2.5)
    xi = white_noise((n, n), g)
    return Workload("antireflect-ar-1025", n, p, truth, psf, xi, 0.02, ANTIREFLECT, AR, 3,
                    alpha0=0.01, mu=1e-3, delta=0.0, iters=50)


WORKLOADS = {
    "plain-fp64-72": lambda: _cfg1(),
    "rect-bccb-512": lambda: _cfg2(1),
    "reflect-dct-512": lambda: _cfg2(2),
    "rect-bccb-geometric-512": lambda: _cfg2(3),
    "rect-bccb-2048": lambda: _cfg3(),
    "antireflect-ar-1025": lambda: _cfg_ar(),
}


def make_workload(name: str) -> Workload:
    return WORKLOADS[name]()


def unrolled_workloads(count: int = 16):
    return _cfg5(count=count)
