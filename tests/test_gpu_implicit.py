"""The implicit state (z = W omega, only omega kept) against the FP64 oracle.

The oracle runs the iteration with the frame coefficients z; z^k = W omega^k
holds exactly because z^0 = 0 and every update of eq. (MLBA2) is W applied to
A^T t, so both states must give the oracle's image within the same bars as the
explicit path: 1e-5 per operator, 1e-4 on the restored image after the full
iteration count.  The soft threshold is continuous, so a coefficient within
round-off of its threshold changes the result by round-off only.
"""
import numpy as np
import pytest

import synth
from oracle import blur as oblur
from oracle import framelet as ofr
from oracle import mlba as omlba
from tests._util import announce, cached, cuda, host, max_err, observed, rel_err, workload_key

pytestmark = pytest.mark.gpu

TOL_L2 = 1e-5
TOL_MAX = 1e-4
TOL_IMAGE = 1e-4


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


@pytest.mark.parametrize("N,L", [(9, 1), (72, 1), (104, 2), (257, 3), (300, 4), (528, 2), (130, 4), (2078, 3)])
def test_shrink_synthesis_operator(mlba, N, L):
    """W^T(delta S_mu(W omega)) against the oracle's synthesis of the thresholded
    analysis, with thresholds that cut a large share of every band."""
    announce(f"shrink synthesis N={N} L={L}")
    g = synth.rng(7000 + N + L)
    omega = synth.shapes_image(N, g, n_rect=8, n_disk=4, n_bumps=4) + 0.05 * g.standard_normal((N, N))
    z = ofr.analysis(omega, L)
    # per-band mu near the band's median magnitude
    mu = np.array([np.median(np.abs(z[b])) for b in range(8 * L + 1)])
    delta = 0.7
    ref = ofr.synthesis(delta * omlba.soft_threshold(z, mu), L)
    with mlba.Plan(N, 1, 2, mlba.NONE, L, cuda(np.ones((1, 1)))) as plan:
        f = host(plan.shrink_synthesis(cuda(omega), mu, delta))
        # the explicit pair on the same input agrees too
        fe = host(plan.threshold_synthesis(plan.analysis(cuda(omega)), mu, delta))
    print(f"  rel {rel_err(f, ref):.2e} max {max_err(f, ref):.2e} vs explicit {rel_err(f, fe):.2e}", flush=True)
    assert rel_err(f, ref) < TOL_L2 and max_err(f, ref) < TOL_MAX
    assert rel_err(f, fe) < TOL_L2


def _schedules(w, iters):
    def compute():
        alphas = omlba.alpha_table(w.alpha_kind, w.alpha0, iters, w.alpha_ratio, w.alpha_floor)
        return alphas, omlba.delta_table(w.psf, w.n, w.bc, w.precond, alphas, w.delta, iters + 1)
    return cached(("schedules",) + workload_key(w, iters), compute)


@pytest.mark.parametrize("name", ["plain-fp64-72", "rect-bccb-512", "reflect-dct-512", "rect-bccb-geometric-512"])
def test_workloads_implicit(mlba, name):
    import dataclasses
    w = synth.make_workload(name)
    if name == "plain-fp64-72":
        w = dataclasses.replace(w, delta=0.0)
    announce(f"implicit restore {name} {w.iters} iterations")
    g, nn = observed(w, oblur)
    alphas, deltas = _schedules(w, w.iters)
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        f, info = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=w.iters,
                               implicit=True)
        f = host(f)
    ref = cached(("mlba",) + workload_key(w, w.iters),
                 lambda: omlba.mlba(g, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, w.iters))
    e, er = rel_err(f, ref["f"]), rel_err(info.rnorm, ref["rnorm"])
    print(f"  image rel err {e:.2e}, rnorm rel err {er:.2e}", flush=True)
    assert info.status == 0 and info.iters_done == w.iters
    assert e < TOL_IMAGE and er < TOL_IMAGE and max_err(f, ref["f"]) < TOL_MAX


@pytest.mark.parametrize("n,p,bc,pc,L", [(96, 17, 0, 0, 2), (96, 17, 1, 1, 3), (192, 11, 3, 0, 2),
                                         (128, 7, 2, 0, 4), (384, 25, 0, 1, 2), (64, 5, 1, 0, 1)])
def test_ragged_and_mixed_models_implicit(mlba, n, p, bc, pc, L):
    announce(f"implicit restore n={n} p={p} bc={bc} pc={pc} L={L}")
    gen = synth.rng(n + p + bc * 7 + pc)
    truth = synth.shapes_image(n + p - 1, gen, n_rect=6, n_disk=3, n_bumps=3)
    H = synth.motion_psf(p, p - 2.0, gen.uniform(0, np.pi))
    g = synth.add_noise(oblur.blur(truth, H, 0), synth.white_noise((n, n), gen), 0.01)
    iters = 40
    alphas = np.full(iters, 0.1)
    d = omlba.delta_auto(omlba.opnorm(H, n, bc, pc, 0.1, tol=1e-6))
    deltas = np.full(iters + 1, d)
    mu = np.linspace(1e-3, 3e-3, 8 * L + 1)
    with mlba.Plan(n, p, bc, pc, L, cuda(H)) as plan:
        f, info = plan.restore(cuda(g), alpha_table=alphas, mu=mu, delta_table=deltas, iters=iters, implicit=True)
        f = host(f)
    ref = omlba.mlba(g, H, bc, pc, L, alphas, deltas, mu, iters)
    assert rel_err(f, ref["f"]) < TOL_IMAGE and max_err(f, ref["f"]) < TOL_MAX
    assert rel_err(info.rnorm, ref["rnorm"]) < TOL_IMAGE


def test_full_size_implicit(mlba):
    """The 2048^2 bench workload, 3 iterations: image and W omega against the
    oracle's image and z."""
    import torch
    w = synth.make_workload("rect-bccb-2048")
    iters = 3
    announce(f"implicit restore rect-bccb-2048 {iters} iterations")
    g, _ = observed(w, oblur)
    alphas = np.full(iters, w.alpha0)
    deltas = np.full(iters + 1, 0.3)
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        om = torch.zeros((plan.N, plan.N), dtype=torch.float32, device="cuda")
        f, info = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=iters, z=om,
                               implicit=True)
        z = host(plan.analysis(om))
        f = host(f)
    ref = omlba.mlba(g, w.psf, w.bc, w.precond, w.levels, alphas, deltas, w.mu, iters)
    print(f"  image {rel_err(f, ref['f']):.2e} state {rel_err(z, ref['z']):.2e}", flush=True)
    assert rel_err(f, ref["f"]) < 1e-5
    assert rel_err(z, ref["z"]) < 1e-5
    assert rel_err(info.rnorm, ref["rnorm"]) < 1e-6


def test_resume_determinism_and_explicit_agreement(mlba):
    import torch
    w = synth.make_workload("plain-fp64-72")
    announce("implicit resume + determinism")
    g, _ = observed(w, oblur)
    it = 12
    alphas = np.full(it, 0.05)
    deltas = np.full(it + 1, 0.25)
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        o1 = torch.zeros((plan.N, plan.N), device="cuda")
        f1, i1 = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=it, z=o1,
                              implicit=True)
        o2 = torch.zeros_like(o1)
        _, ia = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=5, z=o2,
                             implicit=True)
        f2, ib = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=7, k0=5, z=o2,
                              implicit=True)
        f3, i3 = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=it, implicit=True)
        assert torch.equal(o1, o2)
        assert torch.equal(f1, f2) and torch.equal(f1, f3)
        assert i1.rnorm == ia.rnorm + ib.rnorm == i3.rnorm
        fe, _ = plan.restore(cuda(g), alpha_table=alphas, mu=w.mu, delta_table=deltas, iters=it)
        assert rel_err(host(f1), host(fe)) < 1e-5


def test_rejects_bad_state_mode(mlba):
    import ctypes
    from paper_1504_07234_amd import _lib
    announce("state mode check")
    w = synth.make_workload("plain-fp64-72")
    with mlba.Plan(w.n, w.p, w.bc, w.precond, w.levels, cuda(w.psf)) as plan:
        lib = _lib.load()
        prm = _lib.Params()
        mus = (ctypes.c_double * 1)(1e-3)
        prm.alpha.alpha0 = 0.05
        prm.mu = ctypes.cast(mus, _lib.c_dbl_p)
        prm.n_mu = 1
        prm.delta = 0.2
        prm.iters = 1
        prm.state = 2
        g = cuda(np.zeros((w.n, w.n)))
        f = cuda(np.zeros((plan.N, plan.N)))
        st = lib.mlba_restore(plan._h, ctypes.c_void_p(g.data_ptr()), ctypes.byref(prm),
                              ctypes.c_void_p(f.data_ptr()), None, None, None, None)
        assert st == _lib.EINVAL
