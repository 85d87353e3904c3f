"""The benchmarked configuration over a long run against the FP64 oracle.

2048 x 2048 observation, 31 x 31 disk (radius 15), 3 framelet levels, BCCB
preconditioner with alpha = 0.02 (Algorithm 1), the implicit state
(z = W omega), A and A^T on the 2304-point FFT grid (fused with the 2048-point
preconditioner passes) and the library's automatic step (section 3's
convergence theorem, the norm by Lanczos on the GPU): 100 iterations of
eq. (MLBA2), as bench.py times them.  The oracle takes its own automatic step
(ARPACK in FP64) and runs the same 100 iterations with the frame coefficients
z; it prints a line after every block of iterations (the oracle needs
minutes at this size).

Bars: the automatic step within 1e-6, the restored image within 1e-4
(||.||_2-relative and element by element relative to the image's largest
value), the residual-norm history within 1e-4 (as a vector and per entry).
"""
import time

import numpy as np
import pytest

import synth
from oracle import blur as oblur
from oracle import mlba as omlba
from tests._util import announce, cuda, host, max_err, observed, rel_err

pytestmark = pytest.mark.gpu

ITERS = 100
BLOCK = 20


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


def test_full_size_100_iterations(mlba, capsys):
    w = synth.make_workload("rect-bccb-2048")
    assert (w.n, w.p, w.levels, w.alpha0, w.delta) == (2048, 31, 3, 0.02, 0.0)
    announce(f"rect-bccb-2048: {ITERS} iterations, implicit state, FFT grid, automatic step")
    g, nn = observed(w, oblur)
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        plan.set_blur(mlba.BLUR_FFT)
        f, info = plan.restore(cuda(g), alpha=w.alpha0, mu=w.mu, delta=0.0, iters=ITERS, implicit=True)
        f = host(f)
    assert info.status == 0 and info.iters_done == ITERS

    def progress(msg):
        with capsys.disabled():
            print(f"  [oracle] {msg}", flush=True)

    t0 = time.perf_counter()
    deltas = omlba.delta_table(w.psf, w.n, w.bc, w.precond, [w.alpha0], 0.0, ITERS + 1)
    progress(f"automatic step {deltas[0]:.9f} ({time.perf_counter() - t0:.0f} s)")
    alphas = np.full(ITERS, w.alpha0)
    z, rn = None, []
    for k0 in range(0, ITERS, BLOCK):
        ref = omlba.mlba(g, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, BLOCK, z0=z, k0=k0)
        z = ref["z"]
        rn.extend(ref["rnorm"])
        progress(f"iterations {k0 + BLOCK}/{ITERS} ({time.perf_counter() - t0:.0f} s)")
    rn = np.asarray(rn)

    ed = abs(info.deltas[0] / deltas[0] - 1.0)
    e, em = rel_err(f, ref["f"]), max_err(f, ref["f"])
    er = rel_err(info.rnorm, rn)
    erk = float(np.max(np.abs(np.asarray(info.rnorm) / rn - 1.0)))
    print(f"  delta gpu {info.deltas[0]:.9f} oracle {deltas[0]:.9f} (rel {ed:.1e}); image rel {e:.2e} max {em:.2e}; "
          f"rnorm rel {er:.2e} per entry {erk:.2e}; final rnorm {rn[-1]:.4f} (noise {nn:.4f})", flush=True)
    assert all(d == info.deltas[0] for d in info.deltas)
    assert ed <= 1e-6
    assert e < 1e-4 and em < 1e-4
    assert er < 1e-4 and erk < 1e-4
