"""mrmf: mixed-radix matrix-free spin/boson Hamiltonians on MI355X.

The HIP library ``libmrmf.so`` (sources in ``csrc/``, C ABI in ``include/mrmf.h``) applies y = H x
without storing H, drives it with a device-resident Lanczos solver, applies its adjoint and runs
batches of lattices in one persistent launch.  This package is the thin Python binding: ``_lib`` is
the ctypes view of the C ABI and ``plan`` wraps it for torch tensors.
"""
from . import _lib  # noqa: F401

__all__ = ["Plan", "build"]


def __getattr__(name):
    if name == "Plan":
        from .plan import Plan
        return Plan
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
