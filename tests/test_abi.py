"""The C ABI library loads without a GPU and exports every entry point that
include/*.h declares; host-side argument validation answers without
touching a device."""
import ctypes
import os
import re

import pytest

from paper_1504_07234_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(mlba_[A-Za-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("mlba_plan_create", "mlba_restore", "mlba_apply_A", "mlba_apply_At", "mlba_apply_P",
                 "mlba_framelet_analysis", "mlba_framelet_synthesis", "mlba_soft_threshold"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_symbols()) <= set(_lib.SIGNATURES)


def _header_defines(prefix):
    text = open(os.path.join(ROOT, "include", "mlba.h")).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(" + prefix + r"\w*)\s+(\d+)", text)}


def test_phase_and_kernel_tables_match_the_header():
    ph = _header_defines("MLBA_PHASE_")
    assert len(_lib.PHASES) == _header_defines("MLBA_NPHASES")["MLBA_NPHASES"]
    for name, idx in ph.items():
        assert _lib.PHASES[idx] == name[len("MLBA_PHASE_"):].lower()
    ks = _header_defines("MLBA_KERNEL_")
    assert len(_lib.KERNELS) == _header_defines("MLBA_NKERNELS")["MLBA_NKERNELS"] == len(ks)
    for name, idx in ks.items():
        assert _lib.KERNELS[idx] == name[len("MLBA_KERNEL_"):].lower()


def test_status_strings():
    lib = _lib.load()
    assert lib.mlba_status_string(0) == b"ok"
    assert lib.mlba_status_string(-1) == b"invalid argument"
    assert lib.mlba_status_string(-2) == b"unsupported size"
    assert lib.mlba_version() >= 1


@pytest.mark.parametrize("n,p,bc,pc,levels,expect", [
    (64, 8, 0, 0, 1, _lib.EINVAL),        # even PSF side
    (64, 67, 0, 0, 1, _lib.EINVAL),       # PSF larger than the image
    (64, 9, 7, 0, 1, _lib.EINVAL),        # unknown boundary model
    (64, 9, 0, 5, 1, _lib.EINVAL),        # unknown preconditioner
    (64, 9, 0, 0, 0, _lib.EINVAL),        # no framelet level
    (64, 9, 0, 0, 5, _lib.EINVAL),        # too many levels
    (1030, 9, 0, 0, 1, _lib.EUNSUPPORTED),  # 1030 = 2 * 5 * 103: its Bluestein length 2160 exceeds one workgroup
    (125, 9, 0, 0, 1, _lib.EUNSUPPORTED),  # odd: the row passes pair rows
    (600, 9, 4, 3, 1, _lib.EUNSUPPORTED),  # antireflective transform length 1198 = 2 * 599: Bluestein length 2400
    (2049, 9, 4, 3, 1, _lib.EUNSUPPORTED),  # antireflective transform length 4096: beyond one workgroup
    (65, 9, 1, 3, 1, _lib.EUNSUPPORTED),    # the antireflective transform goes with the antireflective model
    (5000, 9, 0, 0, 1, _lib.EUNSUPPORTED),
    (4096, 9, 0, 0, 1, _lib.EUNSUPPORTED),   # beyond the one-workgroup transform
    (256, 51, 0, 0, 1, _lib.EUNSUPPORTED),   # PSF window beyond the blur's LDS tile
])
def test_plan_create_rejects_bad_arguments(n, p, bc, pc, levels, expect):
    """Validation happens before any device call, so it runs on the CPU."""
    lib = _lib.load()
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    st = lib.mlba_plan_create(ctypes.byref(h), n, p, bc, pc, levels, dummy, None)
    assert st == expect
    assert not h.value


def test_null_arguments_rejected():
    lib = _lib.load()
    assert lib.mlba_plan_create(None, 64, 9, 0, 0, 1, ctypes.c_void_p(16), None) == _lib.EINVAL
    assert lib.mlba_apply_A(None, None, None, None) == _lib.EINVAL
    assert lib.mlba_restore(None, None, None, None, None, None, None, None) == _lib.EINVAL
    assert lib.mlba_soft_threshold(None, None, 1, 1, None, 1, 1.0, None) == _lib.EINVAL
    assert lib.mlba_plan_destroy(None) == _lib.EINVAL


@pytest.mark.parametrize("n,p,pc,alpha,expect", [
    (4096, 9, 0, 0.05, _lib.EUNSUPPORTED),  # beyond MLBA_STATIC_MAX_N
    (2050, 9, 1, 0.05, _lib.EUNSUPPORTED),  # 2050 = 2 * 5^2 * 41: no Bluestein form in the static variant
    (98, 9, 0, 0.05, _lib.EUNSUPPORTED),    # 98 = 2 * 7^2
    (126, 9, 0, 0.05, _lib.EUNSUPPORTED),   # 126 = 2 * 3^2 * 7
    (125, 9, 0, 0.05, _lib.EUNSUPPORTED),   # odd
    (256, 9, 2, 0.05, _lib.EUNSUPPORTED),   # no preconditioner
    (256, 9, 3, 0.05, _lib.EUNSUPPORTED),   # antireflective transform
    (256, 8, 0, 0.05, _lib.EINVAL),         # even PSF side
    (8, 9, 0, 0.05, _lib.EINVAL),           # PSF larger than the image
    (256, 9, 0, 0.0, _lib.EINVAL),          # alpha must be positive
])
def test_static_preconditioner_rejects_bad_arguments(n, p, pc, alpha, expect):
    """mlba_apply_P_static validates before any device call."""
    lib = _lib.load()
    d = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert lib.mlba_apply_P_static(d, n, p, pc, d, d, alpha, None) == expect
    assert lib.mlba_apply_P_static(None, 64, 9, 0, d, d, 0.05, None) == _lib.EINVAL
