"""The measurement model of bench.py (host only): the FFT-blur grid rule and
the per-kernel algorithmic bytes / flops / launch counts that the reported
rooflines divide by."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1504_07234_amd import _lib  # noqa: E402


def _smooth_even(m):
    if m % 2:
        return False
    while m % 2 == 0:
        m //= 2
    while m % 3 == 0:
        m //= 3
    return m == 1


@pytest.mark.parametrize("N", [8, 9, 100, 105, 528, 1039, 2048, 2078, 2600, 3072])
def test_fft_grid_is_the_smallest_even_smooth_side(N):
    M = bench.fft_grid(N)
    assert M >= N and _smooth_even(M) and M <= 3072
    assert not any(_smooth_even(m) for m in range(N, M))


def test_fft_grid_of_the_2048_workload():
    assert bench.fft_grid(2078) == 2304


@pytest.mark.parametrize("implicit,fft_blur", [(True, True), (False, True), (True, False), (False, False)])
def test_kernel_model_names_and_launches(implicit, fft_blur):
    """Every modelled kernel is one of the library's profiled kernels, and the
    launch counts per iteration are those of the iteration's sequence
    (3 levels, rectangular model, BCCB preconditioner)."""
    m = bench.kernel_model(2048, 31, 2078, 3, implicit, fft_blur)
    assert set(m) <= set(_lib.KERNELS)
    launches = {k: v["launches"] for k, v in m.items()}
    if implicit:
        assert launches["lowpass_level"] == 1 and launches["shrink_synthesis"] == 3
    else:
        assert launches["synthesis_level"] == 3 and launches["analysis_level"] == 3
    if fft_blur:
        assert launches["fc_cols"] == 2 and launches["fc_residual_precond_rows"] == 1
        assert launches["precond_rows_fc_fwd"] == 1 and launches["fft_cols"] == 1
    else:
        assert launches["conv_blur"] == 1 and launches["conv_blur_t"] == 1
    for v in m.values():
        assert v["bound"] in ("hbm", "alu") and v["bytes"] >= 0 and v["flops"] >= 0


def test_kernel_model_byte_counts():
    """A few closed forms: the direct A^T into omega moves t once and omega
    twice; the shrink-synthesis moves 3 planes per level, 2 at the top."""
    n, N = 2048, 2078
    m = bench.kernel_model(n, 31, N, 3, True, False)
    assert m["conv_blur_t"]["bytes"] == 4 * (n * n + 2 * N * N)
    assert m["conv_blur_t"]["flops"] == 2 * 31 * 31 * n * n
    assert m["shrink_synthesis"]["bytes"] == 4 * N * N * (3 * 3 - 1)
    # at the published peaks (8 TB/s, 157.3 TFLOP/s) its 119 flops per pixel
    # take less time than its bytes; the direct 31 x 31 blur is bound by its taps
    assert m["shrink_synthesis"]["bound"] == "hbm"
    assert m["conv_blur_t"]["bound"] == "alu"


def test_kernel_model_direct_column_pass():
    """The grid's column pass with compiled taps: A reads the N rows of the
    unknown and keeps n, A^T reads n and keeps N, both read the (M/2+1) p
    taps; 4 FMAs (8 flops) per complex tap and output.  Other PSF sizes keep
    the transform pair, which also reads the PSF spectrum."""
    n, N = 2048, 2078
    hm = bench.fft_grid(N) // 2 + 1
    m = bench.kernel_model(n, 31, N, 3, True, True)
    assert bench.direct_cols(31) and not bench.direct_cols(49)
    assert m["fc_cols"]["bytes"] == 2 * 8 * hm * (N + n) + 2 * 8 * hm * 31
    assert m["fc_cols"]["flops"] == 8 * 31 * hm * (N + n)
    m49 = bench.kernel_model(2048, 49, 2096, 3, True, True)
    M49 = bench.fft_grid(2096)
    assert m49["fc_cols"]["bytes"] == 8 * (M49 // 2 + 1) * (2096 + 2048) + 4 * 8 * (M49 // 2 + 1) * M49
