"""Python binding of libmlba: argument marshalling over the C ABI.

PyTorch supplies device memory and the stream; every computation happens in
the HIP kernels behind include/mlba.h.  All tensors must be contiguous
float32 tensors on the current HIP device.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check

RECT, REFLECT, PERIODIC, ZERO, ANTIREFLECT = (_lib.BC_RECT, _lib.BC_REFLECT, _lib.BC_PERIODIC, _lib.BC_ZERO,
                                             _lib.BC_ANTIREFLECT)
BCCB, DCT, NONE, AR = _lib.PRECOND_BCCB, _lib.PRECOND_DCT, _lib.PRECOND_NONE, _lib.PRECOND_AR
MLBA, ALG4, ALG2 = _lib.METHOD_MLBA, _lib.METHOD_ALG4, _lib.METHOD_ALG2
BLUR_DIRECT, BLUR_FFT = _lib.BLUR_DIRECT, _lib.BLUR_FFT


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, name: str, shape=None) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _dbl_array(values):
    arr = (ctypes.c_double * len(values))(*[float(v) for v in values])
    return arr, ctypes.cast(arr, _lib.c_dbl_p)


@dataclass
class RestoreInfo:
    status: int
    iters_done: int
    rnorm: list
    alphas: list = None
    pcg_steps: list = None
    deltas: list = None


class Plan:
    """A restoration plan: sizes, boundary model, preconditioner, framelet
    levels and the PSF (copied to the plan; its spectrum is computed at
    creation)."""

    def __init__(self, n: int, p: int, bc: int, precond: int, levels: int, psf: torch.Tensor, stream=None):
        self._lib = _lib.load()
        self._h = ctypes.c_void_p()
        psf = psf.contiguous()
        check(self._lib.mlba_plan_create(ctypes.byref(self._h), n, p, bc, precond, levels,
                                         _dev(psf, "psf", (p, p)), _stream(stream)), "mlba_plan_create")
        dims = [ctypes.c_int() for _ in range(4)]
        check(self._lib.mlba_plan_dims(self._h, *[ctypes.byref(d) for d in dims]), "mlba_plan_dims")
        self.n, self.p, self.N, self.bands = (d.value for d in dims)
        self.bc, self.precond, self.levels = bc, precond, levels

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if self._h:
            torch.cuda.synchronize()
            self._lib.mlba_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers -----------------------------------------------------------
    def _new(self, *shape):
        return torch.empty(shape, dtype=torch.float32, device="cuda")

    def set_psf(self, psf: torch.Tensor, stream=None):
        psf = psf.contiguous()
        check(self._lib.mlba_plan_set_psf(self._h, _dev(psf, "psf", (self.p, self.p)), _stream(stream)),
              "mlba_plan_set_psf")

    def set_blur(self, mode: int, stream=None):
        """BLUR_DIRECT or BLUR_FFT for A and A^T (rectangular model)."""
        check(self._lib.mlba_plan_set_blur(self._h, int(mode), _stream(stream)), "mlba_plan_set_blur")

    def autotune(self, reps: int = 5, stream=None) -> dict:
        """Times the direct and the FFT blur and keeps the faster (see mlba_plan_autotune)."""
        ms = (ctypes.c_double * 4)()
        mode = check(self._lib.mlba_plan_autotune(self._h, int(reps), ms, _stream(stream)), "mlba_plan_autotune")
        return {"blur": "fft" if mode == _lib.BLUR_FFT else "direct",
                "direct_ms": [ms[0], ms[1]], "fft_ms": [ms[2], ms[3]] if ms[2] >= 0 else None}

    def opnorm(self, alpha: float, iters: int = 1000, stream=None) -> float:
        """||A^T P_alpha A|| (Lanczos, at most `iters` steps; power steps for the
        antireflective model), see mlba_plan_opnorm."""
        out = ctypes.c_double()
        check(self._lib.mlba_plan_opnorm(self._h, float(alpha), int(iters), ctypes.byref(out), _stream(stream)),
              "mlba_plan_opnorm")
        return out.value

    def auto_step(self, alpha: float, stream=None) -> float:
        """The step the library takes for delta <= 0 at a constant alpha (a
        zero-iteration restore that reports its delta_k)."""
        g = torch.zeros((self.n, self.n), dtype=torch.float32, device="cuda")
        _, info = self.restore(g, alpha=alpha, mu=0.0, delta=0.0, iters=0, stream=stream)
        return info.deltas[0]

    # -- operators ---------------------------------------------------------
    def apply_A(self, u, out=None, stream=None):
        out = self._new(self.n, self.n) if out is None else out
        check(self._lib.mlba_apply_A(self._h, _dev(u, "u", (self.N, self.N)), _dev(out, "out", (self.n, self.n)),
                                     _stream(stream)), "mlba_apply_A")
        return out

    def residual(self, g, u, out=None, stream=None):
        out = self._new(self.n, self.n) if out is None else out
        check(self._lib.mlba_residual(self._h, _dev(g, "g", (self.n, self.n)), _dev(u, "u", (self.N, self.N)),
                                      _dev(out, "out", (self.n, self.n)), _stream(stream)), "mlba_residual")
        return out

    def apply_At(self, y, out=None, stream=None):
        out = self._new(self.N, self.N) if out is None else out
        check(self._lib.mlba_apply_At(self._h, _dev(y, "y", (self.n, self.n)), _dev(out, "out", (self.N, self.N)),
                                      _stream(stream)), "mlba_apply_At")
        return out

    def apply_P(self, r, alpha: float, out=None, stream=None):
        out = self._new(self.n, self.n) if out is None else out
        check(self._lib.mlba_apply_P(self._h, _dev(r, "r", (self.n, self.n)), _dev(out, "out", (self.n, self.n)),
                                     float(alpha), _stream(stream)), "mlba_apply_P")
        return out

    def analysis(self, f, out=None, stream=None):
        out = self._new(self.bands, self.N, self.N) if out is None else out
        check(self._lib.mlba_framelet_analysis(self._h, _dev(f, "f", (self.N, self.N)),
                                               _dev(out, "out", (self.bands, self.N, self.N)), _stream(stream)),
              "mlba_framelet_analysis")
        return out

    def analysis_update(self, w, z, stream=None):
        check(self._lib.mlba_analysis_update(self._h, _dev(w, "w", (self.N, self.N)),
                                             _dev(z, "z", (self.bands, self.N, self.N)), _stream(stream)),
              "mlba_analysis_update")
        return z

    def synthesis(self, z, out=None, stream=None):
        out = self._new(self.N, self.N) if out is None else out
        check(self._lib.mlba_framelet_synthesis(self._h, _dev(z, "z", (self.bands, self.N, self.N)),
                                                _dev(out, "out", (self.N, self.N)), _stream(stream)),
              "mlba_framelet_synthesis")
        return out

    def threshold_synthesis(self, z, mu, delta: float, out=None, stream=None):
        out = self._new(self.N, self.N) if out is None else out
        mus = [mu] if isinstance(mu, (int, float)) else list(mu)
        arr, ptr = _dbl_array(mus)
        check(self._lib.mlba_threshold_synthesis(self._h, _dev(z, "z", (self.bands, self.N, self.N)), ptr,
                                                 len(mus), float(delta), _dev(out, "out", (self.N, self.N)),
                                                 _stream(stream)), "mlba_threshold_synthesis")
        return out

    # -- phase timing --------------------------------------------------------
    def apply_CtP(self, r, alpha: float, out=None, stream=None):
        """t = C^T (C C^T + alpha I)^{-1} r (the direction of Algorithm 4)."""
        out = self._new(self.n, self.n) if out is None else out
        check(self._lib.mlba_apply_CtP(self._h, _dev(r, "r", (self.n, self.n)), _dev(out, "out", (self.n, self.n)),
                                       float(alpha), _stream(stream)), "mlba_apply_CtP")
        return out

    def shrink_synthesis(self, omega, mu, delta: float, out=None, stream=None):
        """f = W^T(delta S_mu(W omega)) (the implicit state's synthesis)."""
        out = self._new(self.N, self.N) if out is None else out
        mus = [mu] if isinstance(mu, (int, float)) else list(mu)
        arr, ptr = _dbl_array(mus)
        check(self._lib.mlba_shrink_synthesis(self._h, _dev(omega, "omega", (self.N, self.N)), ptr, len(mus),
                                              float(delta), _dev(out, "out", (self.N, self.N)), _stream(stream)),
              "mlba_shrink_synthesis")
        return out

    def profile_begin(self, max_iters: int, every: int = 1):
        """Record HIP events in the next restorations: every `every`-th iteration, at most `max_iters`."""
        check(self._lib.mlba_profile_begin(self._h, int(max_iters)), "mlba_profile_begin")
        if every != 1:
            check(self._lib.mlba_profile_every(self._h, int(every)), "mlba_profile_every")

    def profile_end(self):
        """{phase: (milliseconds summed, kernel launches)} and the iteration count."""
        ms = (ctypes.c_double * len(_lib.PHASES))()
        launches = (ctypes.c_int * len(_lib.PHASES))()
        iters = ctypes.c_int()
        check(self._lib.mlba_profile_end(self._h, ms, launches, ctypes.byref(iters)), "mlba_profile_end")
        return {ph: (ms[i], launches[i]) for i, ph in enumerate(_lib.PHASES)}, iters.value

    def profile_kernels(self):
        """{kernel: (milliseconds summed, launches)} of the last profile_end (kernels that ran)."""
        ms = (ctypes.c_double * len(_lib.KERNELS))()
        launches = (ctypes.c_int * len(_lib.KERNELS))()
        check(self._lib.mlba_profile_kernels(self._h, ms, launches), "mlba_profile_kernels")
        return {k: (ms[i], launches[i]) for i, k in enumerate(_lib.KERNELS) if launches[i] > 0}

    # -- restoration -------------------------------------------------------
    def restore(self, g, *, alpha=0.05, alpha_kind: int = _lib.ALPHA_CONST, alpha_ratio: float = 1.0,
                alpha_floor: float = 0.0, alpha_table=None, mu=1e-3, delta: float = 0.0, delta_table=None,
                iters: int = 50, k0: int = 0, z=None, out=None, stop=None, track: bool = True,
                implicit: bool = False, method: int = _lib.METHOD_MLBA, ns=None, pcg=None, stream=None):
        """Run `iters` iterations of eq. (MLBA2) (method METHOD_MLBA) or eq. (Alg4)
        (METHOD_ALG4, square models); returns (f, RestoreInfo).

        ns: (q, rho) selects Algorithm 4-NS (alpha_n solved per iteration, alpha is
        the first Newton start; needs stop=(noise_norm, ., .), whose gamma is
        replaced by tau = (1 + 2 rho) / (1 - 2 rho)).  RestoreInfo.alphas holds the
        alpha_k used.
        pcg: (max steps, tolerance) of Algorithm 2 (method ALG2; default (5, 1e-3));
        RestoreInfo.pcg_steps holds beta_n.

        implicit: keep the state as omega (z = W omega, one N x N plane) instead
        of the frame coefficients z.
        z: optional state tensor, [bands, N, N] or [N, N] when implicit (in/out,
        resume with k0).
        stop: optional (noise_norm, gamma, check_every) discrepancy stop.
        track: read back the residual norms (synchronises at the end)."""
        out = self._new(self.N, self.N) if out is None else out
        sched = _lib.AlphaSchedule()
        sched.kind = int(alpha_kind)
        sched.alpha0 = float(alpha)
        sched.ratio = float(alpha_ratio)
        sched.alpha_floor = float(alpha_floor)
        keep = []
        if alpha_table is not None:
            arr, ptr = _dbl_array(alpha_table)
            keep.append(arr)
            sched.kind = _lib.ALPHA_TABLE
            sched.table = ptr
            sched.table_len = len(alpha_table)
        prm = _lib.Params()
        prm.alpha = sched
        mus = [mu] if isinstance(mu, (int, float)) else list(mu)
        marr, mptr = _dbl_array(mus)
        keep.append(marr)
        prm.mu = mptr
        prm.n_mu = len(mus)
        prm.delta = float(delta)
        if delta_table is not None:
            darr, dptr = _dbl_array(delta_table)
            keep.append(darr)
            prm.delta_table = dptr
            prm.delta_table_len = len(delta_table)
        prm.iters = int(iters)
        prm.k0 = int(k0)
        if stop is not None:
            st = _lib.Stop(float(stop[0]), float(stop[1]), int(stop[2]))
            keep.append(st)
            prm.stop = ctypes.pointer(st)
        prm.state = _lib.STATE_IMPLICIT if implicit else _lib.STATE_EXPLICIT
        prm.method = int(method)
        if ns is not None:
            prm.alpha.kind = _lib.ALPHA_NS
            prm.alpha.ns_q, prm.alpha.ns_rho = float(ns[0]), float(ns[1])
        aout = (ctypes.c_double * max(1, iters))() if track else None
        prm.alpha_out = ctypes.cast(aout, _lib.c_dbl_p) if track else None
        if pcg is not None:
            prm.pcg_max, prm.pcg_tol = int(pcg[0]), float(pcg[1])
        bout = (ctypes.c_int * max(1, iters))() if track else None
        prm.pcg_steps_out = ctypes.cast(bout, _lib.c_int_p) if track else None
        dout = (ctypes.c_double * (iters + 1))() if track else None
        prm.delta_out = ctypes.cast(dout, _lib.c_dbl_p) if track else None
        zshape = (self.N, self.N) if implicit else (self.bands, self.N, self.N)
        zp = ctypes.c_void_p() if z is None else _dev(z, "z", zshape)
        rn = (ctypes.c_double * max(1, iters))() if track else None
        done = ctypes.c_int(iters)
        status = self._lib.mlba_restore(self._h, _dev(g, "g", (self.n, self.n)), ctypes.byref(prm),
                                        _dev(out, "out", (self.N, self.N)), zp,
                                        ctypes.cast(rn, _lib.c_dbl_p) if track else None,
                                        ctypes.byref(done) if track else None, _stream(stream))
        check(status, "mlba_restore")
        info = RestoreInfo(status, done.value, list(rn[:done.value]) if track else [],
                           list(aout[:done.value]) if track else [],
                           list(bout[:done.value]) if (track and method == _lib.METHOD_ALG2) else [],
                           list(dout[:done.value + 1]) if track else [])
        return out, info


def soft_threshold(z: torch.Tensor, mu, delta: float = 1.0, out=None, stream=None):
    """x = delta * S_mu(z) over the leading (band) axis of z."""
    lib = _lib.load()
    out = torch.empty_like(z) if out is None else out
    bands = z.shape[0] if z.dim() >= 2 else 1
    elems = z.numel() // bands
    mus = [mu] if isinstance(mu, (int, float)) else list(mu)
    arr, ptr = _dbl_array(mus)
    check(lib.mlba_soft_threshold(_dev(z, "z"), _dev(out, "out", tuple(z.shape)), bands, elems, ptr, len(mus),
                                  float(delta), _stream(stream)), "mlba_soft_threshold")
    return out


def apply_P_static(psf: torch.Tensor, n: int, precond: int, r: torch.Tensor, alpha: float, out=None, stream=None):
    """t = P_alpha r without a plan and without device allocation (see
    mlba_apply_P_static): BCCB or DCT, the PSF's spectrum rebuilt per call."""
    lib = _lib.load()
    p = psf.shape[0]
    out = torch.empty((n, n), dtype=torch.float32, device=r.device) if out is None else out
    check(lib.mlba_apply_P_static(_dev(psf, "psf", (p, p)), int(n), int(p), int(precond), _dev(r, "r", (n, n)),
                                  _dev(out, "out", (n, n)), float(alpha), _stream(stream)), "mlba_apply_P_static")
    return out


class Batch:
    """Many restorations advanced together (one launch per phase covering all
    images), optionally replayed from a captured hipGraph.  The batch uses the
    given plans' workspaces; keep the plans alive and idle while it runs."""

    def __init__(self, plans, max_iters: int, stream=None):
        self._lib = _lib.load()
        self.plans = list(plans)
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        check(self._lib.mlba_batch_create(ctypes.byref(self._h), len(self.plans), arr, int(max_iters),
                                          _stream(stream)), "mlba_batch_create")
        self.max_iters = int(max_iters)

    def close(self):
        if self._h:
            torch.cuda.synchronize()
            self._lib.mlba_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def autotune(self, reps: int = 5, stream=None) -> dict:
        """Times the candidate tile shapes of the tunable phases on this batch and
        keeps the fastest (see mlba_batch_autotune); returns the choices and timings."""
        t = _lib.BatchTuning()
        check(self._lib.mlba_batch_autotune(self._h, int(reps), ctypes.byref(t), _stream(stream)),
              "mlba_batch_autotune")
        return {"conv_rows": list(t.conv_rows), "fft_rows_cap": t.fft_rows_cap, "fft_cols_cap": t.fft_cols_cap,
                "conv_ms": [list(r) for r in t.conv_ms], "rows_ms": list(t.rows_ms), "cols_ms": list(t.cols_ms)}

    def set_tiles(self, conv_rows=(1, 1), fft_rows_cap: int = 0, fft_cols_cap: int = 0, stream=None):
        """Sets the tile shapes directly (see mlba_batch_set_tiles)."""
        t = _lib.BatchTuning()
        t.conv_rows[0], t.conv_rows[1] = int(conv_rows[0]), int(conv_rows[1])
        t.fft_rows_cap, t.fft_cols_cap = int(fft_rows_cap), int(fft_cols_cap)
        check(self._lib.mlba_batch_set_tiles(self._h, ctypes.byref(t), _stream(stream)), "mlba_batch_set_tiles")

    def restore(self, gs, *, alpha, mu=1e-3, delta=None, iters: int = 100, outs=None, zs=None,
                use_graph: bool = True, track: bool = False, implicit: bool = False, stream=None):
        """Returns (list of restored images, residual norms [count][iters] or None).
        implicit: keep omega (z = W omega, zs [N, N] per image) instead of z."""
        count = len(self.plans)
        if len(gs) != count:
            raise ValueError("one observed image per plan")
        outs = [self.plans[i]._new(self.plans[i].N, self.plans[i].N) for i in range(count)] if outs is None else outs
        gp = (ctypes.c_void_p * count)(*[_dev(g, "g", (p.n, p.n)).value for g, p in zip(gs, self.plans)])
        fp = (ctypes.c_void_p * count)(*[_dev(f, "f", (p.N, p.N)).value for f, p in zip(outs, self.plans)])
        zp = None
        if zs is not None:
            zp = (ctypes.c_void_p * count)(*[_dev(z, "z", (p.N, p.N) if implicit else (p.bands, p.N, p.N)).value
                                             for z, p in zip(zs, self.plans)])
        alphas = [alpha] * count if isinstance(alpha, (int, float)) else list(alpha)
        deltas = [0.0] * count if delta is None else ([delta] * count if isinstance(delta, (int, float)) else list(delta))
        if isinstance(mu, (int, float)):
            mus, n_mu = [mu] * count, 1
        else:
            rows = [list(m) if hasattr(m, "__len__") else [m] for m in mu]
            n_mu = len(rows[0])
            mus = [v for r in rows for v in r]
        aarr, ap = _dbl_array(alphas)
        marr, mp = _dbl_array(mus)
        darr, dp = _dbl_array(deltas)
        rn = (ctypes.c_double * (count * max(iters, 1)))() if track else None
        st = self._lib.mlba_batch_restore(self._h, gp, ap, mp, n_mu, dp, int(iters), fp, zp,
                                          ctypes.cast(rn, _lib.c_dbl_p) if track else None,
                                          _lib.STATE_IMPLICIT if implicit else _lib.STATE_EXPLICIT,
                                          int(bool(use_graph)), _stream(stream))
        check(st, "mlba_batch_restore")
        norms = None
        if track:
            norms = [list(rn[i * iters:(i + 1) * iters]) for i in range(count)]
        return outs, norms


class Unrolled:
    """K unrolled iterations of eq. (MLBA2) for a batch of images (rectangular
    blur, BCCB preconditioner, one shared PSF, alpha, mu and delta) and their
    reverse-mode gradient, checkpointing z every `ckpt_every` iterations.
    Owns one plan per image."""

    def __init__(self, sizes, p: int, levels: int, psf: torch.Tensor, iters: int, ckpt_every: int = 5,
                 stream=None):
        self._lib = _lib.load()
        self.sizes = [int(n) for n in sizes]
        self.p, self.levels, self.iters, self.ckpt_every = int(p), int(levels), int(iters), int(ckpt_every)
        self.plans = [Plan(n, p, RECT, BCCB, levels, psf, stream) for n in self.sizes]
        self.bands = self.plans[0].bands
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_void_p * len(self.plans))(*[pl._h.value for pl in self.plans])
        check(self._lib.mlba_unrolled_create(ctypes.byref(self._h), len(self.plans), arr, self.iters,
                                             self.ckpt_every, _stream(stream)), "mlba_unrolled_create")
        seg = ctypes.c_int()
        elems = (ctypes.c_size_t * len(self.plans))()
        check(self._lib.mlba_unrolled_dims(self._h, ctypes.byref(seg), elems), "mlba_unrolled_dims")
        self.segments = seg.value
        self.ckpt_elems = list(elems)

    def close(self):
        if self._h:
            torch.cuda.synchronize()
            self._lib.mlba_unrolled_destroy(self._h)
            self._h = ctypes.c_void_p()
        for pl in getattr(self, "plans", []):
            pl.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_psf(self, psf: torch.Tensor, stream=None):
        for pl in self.plans:
            pl.set_psf(psf, stream)

    def _ptrs(self, ts, name, shape_of):
        if len(ts) != len(self.plans):
            raise ValueError(f"{name}: one tensor per image")
        return (ctypes.c_void_p * len(ts))(*[_dev(t, name, shape_of(pl)).value for t, pl in zip(ts, self.plans)])

    def _mu(self, mu):
        mus = [float(mu)] if isinstance(mu, (int, float)) else [float(v) for v in mu]
        return _dbl_array(mus) + (len(mus),)

    def new_checkpoints(self):
        dev = torch.device("cuda", torch.cuda.current_device())
        return [torch.empty(e, device=dev, dtype=torch.float32) for e in self.ckpt_elems]

    def forward(self, gs, *, alpha: float, mu, delta: float, ckpts=None, outs=None, stream=None):
        """Returns (list of f_i, list of checkpoint buffers)."""
        ckpts = self.new_checkpoints() if ckpts is None else ckpts
        outs = [pl._new(pl.N, pl.N) for pl in self.plans] if outs is None else outs
        gp = self._ptrs(gs, "g", lambda pl: (pl.n, pl.n))
        fp = self._ptrs(outs, "f", lambda pl: (pl.N, pl.N))
        cp = (ctypes.c_void_p * len(ckpts))(*[_dev(c, "ckpt", (e,)).value for c, e in zip(ckpts, self.ckpt_elems)])
        marr, mp, n_mu = self._mu(mu)
        check(self._lib.mlba_unrolled_forward(self._h, gp, float(alpha), mp, n_mu, float(delta), cp, fp,
                                              _stream(stream)), "mlba_unrolled_forward")
        return outs, ckpts

    def backward(self, gs, dfs, ckpts, *, alpha: float, mu, delta: float, want_dg: bool = True, stream=None):
        """Gradients of a loss with dl/df_i = dfs[i]: dict with 'mu' (bands,),
        'alpha' (), 'psf' (p, p) float64 device tensors and 'g' (list of
        n_i x n_i float32, or None)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        gp = self._ptrs(gs, "g", lambda pl: (pl.n, pl.n))
        dp = self._ptrs(dfs, "df", lambda pl: (pl.N, pl.N))
        cp = (ctypes.c_void_p * len(ckpts))(*[_dev(c, "ckpt", (e,)).value for c, e in zip(ckpts, self.ckpt_elems)])
        dmu = torch.empty(self.bands, device=dev, dtype=torch.float64)
        dal = torch.empty((), device=dev, dtype=torch.float64)
        dpsf = torch.empty(self.p, self.p, device=dev, dtype=torch.float64)
        dgs = [pl._new(pl.n, pl.n) for pl in self.plans] if want_dg else None
        dgp = self._ptrs(dgs, "dg", lambda pl: (pl.n, pl.n)) if want_dg else None
        marr, mp, n_mu = self._mu(mu)
        check(self._lib.mlba_unrolled_backward(self._h, gp, float(alpha), mp, n_mu, float(delta), cp, dp,
                                               ctypes.c_void_p(dmu.data_ptr()), ctypes.c_void_p(dal.data_ptr()),
                                               ctypes.c_void_p(dpsf.data_ptr()), dgp, _stream(stream)),
              "mlba_unrolled_backward")
        return {"mu": dmu, "alpha": dal, "psf": dpsf, "g": dgs}


class UnrolledMLBA(torch.autograd.Function):
    """f = unrolled MLBA(g; psf, alpha, mu) over a batch of equal-size images.

    g: (B, n, n) float32; psf: (p, p) float32; alpha: 0-d tensor; mu: (bands,)
    tensor; returns f: (B, N, N).  `engine` is an Unrolled built for B images
    of side n (its PSF is replaced by `psf` on every call); delta is a float.
    The backward pass recomputes each checkpoint segment once."""

    @staticmethod
    def forward(ctx, g, psf, alpha, mu, engine, delta):
        B = g.shape[0]
        g = g.detach().contiguous()
        psf_d = psf.detach().contiguous()
        engine.set_psf(psf_d)
        a = float(alpha)
        m = [float(v) for v in mu.detach().reshape(-1).cpu()]
        N = engine.plans[0].N
        f = torch.empty(B, N, N, device=g.device, dtype=torch.float32)
        outs, ckpts = engine.forward([g[i] for i in range(B)], alpha=a, mu=m, delta=delta,
                                     outs=[f[i] for i in range(B)])
        ctx.engine, ctx.delta, ctx.alpha, ctx.mu, ctx.ckpts = engine, delta, a, m, ckpts
        ctx.save_for_backward(g, psf_d)
        return f

    @staticmethod
    def backward(ctx, df):
        g, psf = ctx.saved_tensors
        engine = ctx.engine
        engine.set_psf(psf)
        B = g.shape[0]
        df = df.contiguous()
        res = engine.backward([g[i] for i in range(B)], [df[i] for i in range(B)], ctx.ckpts, alpha=ctx.alpha,
                              mu=ctx.mu, delta=ctx.delta, want_dg=ctx.needs_input_grad[0])
        dg = torch.stack(res["g"]) if res["g"] is not None else None
        return (dg, res["psf"].to(psf.dtype), res["alpha"].to(torch.float32), res["mu"].to(torch.float32),
                None, None)


def unrolled_mlba(g, psf, alpha, mu, engine: Unrolled, delta: float):
    """Differentiable K-iteration MLBA restoration (see UnrolledMLBA)."""
    return UnrolledMLBA.apply(g, psf, alpha, mu, engine, delta)
