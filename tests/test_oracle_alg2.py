"""Pins of the Algorithm 2 oracle (section 4.2): the PCG direction against
dense linear algebra (exact solve, the Krylov energy-norm minimiser), the case
where the preconditioner is exact, and the resulting iteration against the
MLBA oracle in that case."""
import numpy as np
import pytest

import synth
from oracle import alg2 as oa2
from oracle import blur as ob
from oracle import mlba as om
from oracle import precond as opc


def _dense(H, n, bc):
    N = ob.unknown_side(n, H.shape[0], bc)
    M = np.zeros((n * n, N * N))
    for j in range(N * N):
        e = np.zeros(N * N)
        e[j] = 1.0
        M[:, j] = ob.blur_direct(e.reshape(N, N), H, bc).ravel()
    return M


def _psf(p, seed):
    g = synth.rng(seed)
    H = g.random((p, p)) + 0.1
    return H / H.sum()


@pytest.mark.parametrize("bc,kind", [(ob.RECT, opc.BCCB), (ob.REFLECT, opc.DCT), (ob.ZERO, opc.BCCB)])
def test_pcg_converges_to_the_solve(bc, kind):
    n, p, alpha = 8, 3, 0.05
    H = _psf(p, 5 + bc)
    r = synth.rng(1).standard_normal((n, n))
    t, steps = oa2.pcg_direction(r, H, bc, kind, alpha, beta_max=200, tol=1e-13)
    A = _dense(H, n, bc)
    ref = np.linalg.solve(A @ A.T + alpha * np.eye(n * n), r.ravel())
    assert steps < 200
    assert np.allclose(t.ravel(), ref, atol=1e-10)


def test_exact_preconditioner_needs_one_step():
    """Periodic model with the BCCB preconditioner: M = A A^T + alpha I, so one
    PCG step is the exact solve and meets any tolerance."""
    n, p, alpha = 10, 5, 0.1
    H = _psf(p, 9)
    r = synth.rng(2).standard_normal((n, n))
    t, steps = oa2.pcg_direction(r, H, ob.PERIODIC, opc.BCCB, alpha, beta_max=5, tol=1e-10)
    assert steps == 1
    assert np.allclose(t, opc.apply_bccb(r, H, alpha), atol=1e-12)


@pytest.mark.parametrize("j", [1, 2, 3])
def test_pcg_step_is_the_krylov_energy_minimiser(j):
    """After j steps, t = M^{-1/2} y_j with y_j the energy-norm minimiser of the
    symmetrised system over K_j (eq. psys), computed densely."""
    n, p, alpha = 8, 3, 0.05
    H = _psf(p, 21)
    bc, kind = ob.RECT, opc.BCCB
    r = synth.rng(3).standard_normal((n, n))
    t, steps = oa2.pcg_direction(r, H, bc, kind, alpha, beta_max=j, tol=0.0)
    assert steps == j
    A = _dense(H, n, bc)
    Bm = A @ A.T + alpha * np.eye(n * n)
    # M from the preconditioner oracle applied to unit vectors
    Minv = np.stack([opc.apply(e.reshape(n, n), H, alpha, kind).ravel() for e in np.eye(n * n)], axis=1)
    w, V = np.linalg.eigh(0.5 * (Minv + Minv.T))
    Mmh = V @ np.diag(np.sqrt(w)) @ V.T  # M^{-1/2}
    K = Mmh @ Bm @ Mmh
    v = Mmh @ r.ravel()
    basis = [v]
    for _ in range(j - 1):
        basis.append(K @ basis[-1])
    Q, _ = np.linalg.qr(np.stack(basis, axis=1))
    y = Q @ np.linalg.solve(Q.T @ K @ Q, Q.T @ v)
    assert np.allclose(t.ravel(), Mmh @ y, atol=1e-10)


def test_alg2_equals_mlba_when_the_preconditioner_is_exact():
    n, p, L, it = 16, 5, 1, 8
    H = _psf(p, 31)
    g = synth.rng(4).standard_normal((n, n))
    alphas = np.full(it, 0.05)
    deltas = np.full(it + 1, 0.5)
    a2 = oa2.alg2(g, H, ob.PERIODIC, opc.BCCB, L, alphas, deltas, 1e-3, it)
    m = om.mlba(g, H, ob.PERIODIC, opc.BCCB, L, alphas, deltas, 1e-3, it)
    assert np.all(a2["betas"] == 1)
    assert np.allclose(a2["f"], m["f"], atol=1e-10)
    assert np.allclose(a2["rnorm"], m["rnorm"], rtol=1e-10)
