"""Example 3's shape (section 6): a 196 x 196 field of view, antireflective
conditions, a PSF that is not quadrantally symmetric.  196 = 2^2 7^2 and the
antireflective transform length 2 * 195 = 390 = 2 * 3 * 5 * 13 both need the
Bluestein form of the transforms.  Table 3's MLBA configurations (Alg-BC3,
Alg-BC1, Alg-Rect1, Alg-Rect3) against the FP64 oracle with its automatic
step, Alg-BC4 (Algorithm 4 with the BCCB matrix) and Alg-Rect2 (Algorithm
2); bar 1e-4 on the restored image and the residual norms.

The scene is a synthetic stand-in for the Boat image, and the PSF a 31-tap
motion blur (the LDS window of the direct blur takes p <= 49)."""
import numpy as np
import pytest

import synth
from oracle import blur as ob
from oracle import mlba as omlba
from oracle import precond as opc
from tests._util import announce, cuda, host, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


@pytest.fixture(scope="module")
def scene():
    n, p = 196, 31
    g0 = synth.rng(196)
    truth = synth.shapes_image(n + p - 1, g0, n_rect=8, n_disk=4, n_bumps=3)
    H = synth.motion_psf(p, p - 4.0, 0.6)
    g = synth.add_noise(ob.blur(truth, H, ob.RECT), synth.white_noise((n, n), g0), 0.01)
    return n, p, H, g


# (name, boundary model, preconditioner, alpha of Table 3)
CONFIGS = [("Alg-BC3", ob.ANTIREFLECT, opc.AR, 0.022), ("Alg-BC1", ob.ANTIREFLECT, opc.BCCB, 0.37),
           ("Alg-Rect1", ob.RECT, opc.BCCB, 0.03), ("Alg-Rect3", ob.RECT, opc.DCT, 0.03)]


@pytest.mark.parametrize("name,bc,pc,alpha", CONFIGS)
def test_example3_shape(mlba, scene, name, bc, pc, alpha):
    n, p, H, g = scene
    iters, L, mu = 15, 2, 1e-3
    announce(f"Example 3 shape {name} n={n} p={p}")
    delta = omlba.delta_auto(omlba.opnorm(H, n, bc, pc, alpha, tol=1e-6))
    ref = omlba.mlba(g, H, bc, pc, L, np.full(iters, alpha), np.full(iters + 1, delta), mu, iters)
    with mlba.Plan(n, p, bc, pc, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=mu, delta=delta, iters=iters, implicit=True)
        f = host(f)
    e = rel_err(f, ref["f"])
    print(f"  delta {delta:.4f} image {e:.2e} rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


def test_example3_alg_bc4(mlba, scene):
    """Alg-BC4 on the same shape: Algorithm 4 (section 5), the direction
    C^T (C C^T + alpha I)^{-1} r with the BCCB matrix of the PSF (FFTs of
    length 196 in the Bluestein form) on the antireflective model, step 1."""
    from oracle import alg4 as oa4
    n, p, H, g = scene
    iters, L, alpha = 15, 2, 0.1
    mu = np.full(8 * L + 1, 1e-3)
    announce(f"Example 3 shape Alg-BC4 n={n} p={p}")
    ref = oa4.alg4(g, H, ob.ANTIREFLECT, opc.BCCB, L, np.full(iters, alpha), np.ones(iters + 1), mu, iters)
    with mlba.Plan(n, p, mlba.ANTIREFLECT, mlba.BCCB, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=mu, delta=1.0, iters=iters, method=mlba.ALG4,
                               implicit=True)
        f = host(f)
    e = rel_err(f, ref["f"])
    print(f"  image {e:.2e} rnorm {rel_err(info.rnorm, ref['rnorm']):.2e}", flush=True)
    assert e < 1e-4
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-4


def test_example3_alg_rect2(mlba, scene):
    """Alg-Rect2 on the same shape: Algorithm 2 (section 4.2), PCG on
    A A^T + alpha I preconditioned by the BCCB matrix (Bluestein-form FFTs of
    length 196), at most 5 PCG steps with a tolerance every iteration misses
    (5 steps each time, so no step count sits near its threshold)."""
    from oracle import alg2 as oa2
    n, p, H, g = scene
    iters, L, alpha, delta, pcg = 10, 2, 0.03, 1.0, (5, 1e-4)
    announce(f"Example 3 shape Alg-Rect2 n={n} p={p}")
    ref = oa2.alg2(g, H, ob.RECT, opc.BCCB, L, np.full(iters, alpha), np.full(iters + 1, delta), 1e-3, iters,
                   beta_max=pcg[0], tol=pcg[1])
    with mlba.Plan(n, p, mlba.RECT, mlba.BCCB, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha=alpha, mu=1e-3, delta=delta, iters=iters, method=mlba.ALG2, pcg=pcg)
        f = host(f)
    e = rel_err(f, ref["f"])
    print(f"  betas {info.pcg_steps}; image {e:.2e}", flush=True)
    assert info.pcg_steps == ref["betas"].tolist() == [pcg[0]] * iters
    assert e < 1e-4
