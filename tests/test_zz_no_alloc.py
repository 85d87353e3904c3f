"""mlba_apply_P_static: the preconditioner without a plan and without device
allocation, against mlba_apply_P of a plan built for the same PSF (the same
kernels; the tables come from the static scratch instead of the plan) and
against the FP64 oracle.  Two calls in a row, the second on a smaller image,
share the one static array; the device's free memory does not move across
calls once the library is loaded.
"""
import numpy as np
import pytest

import synth
from oracle import precond as opc
from tests._util import announce, cuda, host, max_err, rel_err

pytestmark = pytest.mark.gpu

TOL_L2 = 1e-5   # the per-operator bar against the oracle
TOL_MAX = 1e-4


@pytest.fixture(scope="module")
def mlba():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_07234_amd import mlba as m
    return m


def _case(n, p, seed):
    g = synth.rng(seed)
    H = synth.gaussian_psf(p, g.uniform(1.0, 4.0)) if seed % 2 else synth.motion_psf(p, p - 2.0, g.uniform(0, np.pi))
    r = synth.shapes_image(n, g, n_rect=5, n_disk=3) + 0.1 * g.standard_normal((n, n))
    return H, r


@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("sizes", [((512, 17), (256, 9)), ((2048, 31), (96, 15)), ((160, 11), (120, 7))])
def test_static_matches_plan_twice(mlba, precond, sizes):
    import torch
    ref_oracle = opc.apply_bccb if precond == 0 else opc.apply_dct
    for call, (n, p) in enumerate(sizes):
        announce(f"apply_P_static precond={precond} n={n} p={p} call {call + 1}")
        H, r = _case(n, p, 100 * n + p + precond)
        alpha = 0.03 + 0.01 * call
        Hd, rd = cuda(H), cuda(r)
        t_static = mlba.apply_P_static(Hd, n, precond, rd, alpha)
        with mlba.Plan(n, p, 1 if precond == 1 else 0, precond, 1, Hd) as plan:
            t_plan = plan.apply_P(rd, alpha)
            torch.cuda.synchronize()
            a, b = host(t_static), host(t_plan)
        ref = ref_oracle(r, H, alpha)
        print(f"  vs plan: rel {rel_err(a, b):.1e} max {max_err(a, b):.1e} (identical {np.array_equal(a, b)}); "
              f"vs oracle: rel {rel_err(a, ref):.1e} max {max_err(a, ref):.1e}", flush=True)
        assert rel_err(a, b) <= 1e-6 and max_err(a, b) <= 1e-5
        assert rel_err(a, ref) < TOL_L2 and max_err(a, ref) < TOL_MAX


def test_static_in_place_and_no_allocation(mlba):
    import torch
    n, p = 384, 13
    announce(f"apply_P_static in place n={n}")
    H, r = _case(n, p, 77)
    Hd = cuda(H)
    rd = cuda(r)
    expect = host(mlba.apply_P_static(Hd, n, 0, rd, 0.05))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        mlba.apply_P_static(Hd, n, 0, rd, 0.05, out=rd)  # r and t alias
        rd.copy_(cuda(r))
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    got = host(mlba.apply_P_static(Hd, n, 0, rd, 0.05, out=rd))
    assert np.array_equal(got, expect)


def test_static_rejects(mlba):
    from paper_1504_07234_amd import _lib
    announce("apply_P_static argument errors")
    H = cuda(synth.gaussian_psf(9, 2.0))
    for n, precond, code in ((4096, 0, _lib.EUNSUPPORTED), (2050, 0, _lib.EUNSUPPORTED), (98, 0, _lib.EUNSUPPORTED),
                             (256, 2, _lib.EUNSUPPORTED), (256, 3, _lib.EUNSUPPORTED), (6, 0, _lib.EINVAL)):
        r = cuda(np.zeros((n, n)))
        with pytest.raises(_lib.MLBAError) as ei:
            mlba.apply_P_static(H, n, precond, r, 0.05)
        assert ei.value.status == code, (n, precond)
    r = cuda(np.zeros((64, 64)))
    with pytest.raises(_lib.MLBAError) as ei:
        mlba.apply_P_static(H, 64, 0, r, 0.0)
    assert ei.value.status == _lib.EINVAL
