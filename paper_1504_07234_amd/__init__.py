"""MI355X (gfx950) implementation of preconditioned MLBA frame-based deblurring.

The computation lives in HIP kernels behind the C ABI of include/mlba.h
(libmlba.so, built in-tree by ``python -m paper_1504_07234_amd.build``);
:mod:`paper_1504_07234_amd.mlba` marshals torch tensors onto it.
"""
from ._lib import LIB_PATH, load  # noqa: F401

__all__ = ["LIB_PATH", "load"]
