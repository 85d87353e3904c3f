"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np

import synth


def announce(msg: str):
    """Name the case before any GPU work so a failing run says which one."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def rel_err(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def max_err(a, b) -> float:
    """max |a - b| relative to max |b| (element by element)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def cuda(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().double().numpy()


def observed(w, oracle_blur):
    """g = A f_true + eta for workload ``w`` with the rectangular blur of the
    oracle (the physical model: the scene extends beyond the field of view)."""
    b = oracle_blur.blur(w.truth, w.psf, oracle_blur.RECT)
    return synth.add_noise(b, w.xi, w.noise_level), synth.noise_norm(b, w.noise_level)


def unknown_init(w):
    """The true image restricted to the unknown grid of the workload's model."""
    if w.bc == 0:
        return w.truth
    c = (w.p - 1) // 2
    return w.truth[c:c + w.n, c:c + w.n]


_CACHE = {}


def cached(key, compute):
    """compute() once per test process for `key` (several tests compare the GPU
    against the same oracle run; the cached value is shared, never modified)."""
    if key not in _CACHE:
        _CACHE[key] = compute()
    return _CACHE[key]


def workload_key(w, iters):
    """Everything that fixes a synthetic workload's oracle run: its name (the
    seeded inputs), its schedule parameters and the iteration count."""
    return (w.name, w.alpha_kind, w.alpha0, w.alpha_ratio, w.alpha_floor, w.delta, iters)
