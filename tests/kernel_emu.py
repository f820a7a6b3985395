"""CPU emulation of the plan-specialized kernels (test infrastructure).

The library generates a HIP kernel per plan (mrmf_plan_kernel_source, host only).  Here that source is
compiled for x86 with clang against tests/emu/hip_emu.h and run on host threads, so its indexing,
LDS use and buffer offsets can be checked on the CPU: every buffer access that is not masked off is
verified to lie inside x or y, and the result is compared with the oracle by the tests.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import re
import subprocess
import tempfile

import numpy as np

from paper_2606_02169_amd import _lib as L
from tests.helpers import host_plan

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
CLANG = "/opt/rocm/llvm/bin/clang++"
CACHE = os.path.join(tempfile.gettempdir(), "mrmf_emu_cache")


TUNING = {"schedule": L.MRMF_TUNE_SCHEDULE, "branch_skip": L.MRMF_TUNE_BRANCH_SKIP,
          "load_group": L.MRMF_TUNE_LOAD_GROUP, "blocks_per_cu": L.MRMF_TUNE_BLOCKS_PER_CU,
          "variant": L.MRMF_TUNE_VARIANT, "addressing": L.MRMF_TUNE_ADDRESSING,
          "far_loads": L.MRMF_TUNE_FAR_LOADS, "outer_first": L.MRMF_TUNE_OUTER_FIRST,
          "unroll_top": L.MRMF_TUNE_UNROLL_TOP, "far_dir": L.MRMF_TUNE_FAR_DIR}


def kernel_source(model, dtype: int, inner: int = 0, unrolled: int = -1, require_hermitian=True,
                  tuning=None) -> str | None:
    st, h = host_plan(model, require_hermitian=require_hermitian)
    assert st == 0, st
    try:
        L.call("mrmf_plan_set_kernel", h, L.MRMF_KERNEL_SPECIALIZED, int(inner), int(unrolled))
        for k, v in (tuning or {}).items():
            L.call("mrmf_plan_set_tuning", h, TUNING[k], int(v))
        n = ctypes.c_size_t()
        s = L.lib().mrmf_plan_kernel_source(h, dtype, None, 0, ctypes.byref(n))
        if s != 0:
            return None
        buf = ctypes.create_string_buffer(n.value + 1)
        L.call("mrmf_plan_kernel_source", h, dtype, buf, n.value + 1, ctypes.byref(n))
        return buf.value.decode()
    finally:
        L.lib().mrmf_plan_destroy(h)


def _compile(src: str) -> ctypes.CDLL:
    os.makedirs(CACHE, exist_ok=True)
    key = hashlib.sha256((src + open(os.path.join(EMU, "hip_emu.h")).read()
                          + open(os.path.join(EMU, "emu_driver.cpp")).read()).encode()).hexdigest()[:20]
    so = os.path.join(CACHE, f"k_{key}.so")
    if not os.path.exists(so):
        gen = os.path.join(CACHE, f"k_{key}.cpp")
        with open(gen, "w") as f:
            f.write(src)
        tmp = so + f".tmp{os.getpid()}"
        cmd = [CLANG, "-std=c++17", "-O1", "-pthread", "-fPIC", "-shared", "-w", "-I", EMU,
               "-include", os.path.join(EMU, "hip_emu.h"), "-x", "c++", gen,
               os.path.join(EMU, "emu_driver.cpp"), "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"emulator build failed:\n{r.stderr[:4000]}")
        os.replace(tmp, so)
    lib = ctypes.CDLL(so)
    lib.emu_run.restype = ctypes.c_int
    lib.emu_run.argtypes = [ctypes.c_uint, ctypes.c_uint, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                            ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t]
    lib.emu_run_range.restype = ctypes.c_int
    lib.emu_run_range.argtypes = lib.emu_run.argtypes + [ctypes.c_uint, ctypes.c_uint]
    lib.emu_run_grad.restype = ctypes.c_int
    lib.emu_run_grad.argtypes = [ctypes.c_uint, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    lib.emu_run_sector.restype = ctypes.c_int
    lib.emu_run_sector.argtypes = [ctypes.c_uint, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t]
    lib.emu_run_cheb.restype = ctypes.c_int
    lib.emu_run_cheb.argtypes = ([ctypes.c_uint, ctypes.c_uint, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_double] * 5
                                 + [ctypes.c_uint, ctypes.c_uint])
    lib.emu_run_sector_cheb.restype = ctypes.c_int
    lib.emu_run_sector_cheb.argtypes = ([ctypes.c_uint, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_double] * 5
                                        + [ctypes.c_void_p, ctypes.c_size_t])
    return lib


def launch_shape(src: str):
    block = int(re.search(r"__launch_bounds__\((\d+)\)", src).group(1))
    tiles = int(re.search(r"(\d+) super-tiles", src).group(1))
    return block, tiles


def run(model, x: np.ndarray, theta=None, inner: int = 0, unrolled: int = -1, grid: int | None = None,
        require_hermitian=True, tuning=None, blocks=None) -> np.ndarray:
    """y = H x with the generated kernel, emulated on the CPU."""
    f32 = x.dtype == np.complex64
    src = kernel_source(model, L.MRMF_DTYPE_C if f32 else L.MRMF_DTYPE_Z, inner, unrolled,
                        require_hermitian=require_hermitian, tuning=tuning)
    if src is None:
        raise ValueError("the plan does not qualify for the specialized kernel")
    block, tiles = launch_shape(src)
    if grid is None:
        grid = min(tiles, 8)
    lib = _compile(src)
    th = np.ascontiguousarray(model.theta if theta is None else theta,
                              dtype=np.float32 if f32 else np.float64)
    xx = np.ascontiguousarray(x)
    y = np.full_like(xx, np.nan)
    b0, b1 = blocks if blocks is not None else (0, 0)
    rc = lib.emu_run_range(grid, block, th.ctypes.data, th.nbytes, xx.ctypes.data, xx.nbytes, y.ctypes.data,
                           y.nbytes, b0, b1)
    if rc != 0:
        raise RuntimeError(f"emu_run failed: {rc}")
    return y


def run_cheb(model, x: np.ndarray, prev: np.ndarray, acc: np.ndarray, ea: float, eb: float, eg: float, c: complex,
             inner: int = 0, unrolled: int = -1, grid: int | None = None, tuning=None, blocks=None):
    """The Chebyshev-step kernel (c128): returns (prev', acc') with prev' = ea H x + eb x + eg prev and
    acc' = acc + c prev', emulated on the CPU (rows outside the emulated blocks keep their inputs)."""
    src = kernel_source(model, L.MRMF_SOURCE_CHEB, inner, unrolled, tuning=tuning)
    if src is None:
        raise ValueError("the plan does not qualify for the specialized kernel")
    block, tiles = launch_shape(src)
    if grid is None:
        grid = min(tiles, 8)
    lib = _compile(src)
    th = np.ascontiguousarray(model.theta, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.complex128)
    pv = np.array(prev, dtype=np.complex128, copy=True)
    av = np.array(acc, dtype=np.complex128, copy=True)
    b0, b1 = blocks if blocks is not None else (0, 0)
    rc = lib.emu_run_cheb(grid, block, th.ctypes.data, th.nbytes, xx.ctypes.data, xx.nbytes, pv.ctypes.data,
                          av.ctypes.data, ea, eb, eg, c.real, c.imag, b0, b1)
    if rc != 0:
        raise RuntimeError(f"emu_run_cheb failed: {rc}")
    return pv, av


def run_grad(model, x: np.ndarray, g: np.ndarray, grid: int):
    """The adjoint kernel generated for the plan (c128), emulated on the CPU: (grad_x = H g, per-block
    partial sums [grid][n_params] whose column sums are Re <g | h_p x>)."""
    src = kernel_source(model, L.MRMF_SOURCE_GRAD)
    if src is None:
        raise ValueError("the plan does not qualify for the generated adjoint kernel")
    lib = _compile(src)
    th = np.ascontiguousarray(model.theta, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.complex128)
    gg = np.ascontiguousarray(g, dtype=np.complex128)
    gx = np.full_like(xx, np.nan)
    part = np.full((grid, len(model.theta)), np.nan)
    rc = lib.emu_run_grad(grid, th.ctypes.data, th.nbytes, xx.ctypes.data, xx.nbytes, gg.ctypes.data, gx.ctypes.data,
                          part.ctypes.data, part.nbytes)
    if rc != 0:
        raise RuntimeError(f"emu_run_grad failed: {rc}")
    return gx, part


def sector_source(model, digit_sum: int, dtype: int, tuning=None) -> str | None:
    st, h = host_plan(model)
    assert st == 0, st
    s = ctypes.c_void_p()
    try:
        for k, v in (tuning or {}).items():
            L.call("mrmf_plan_set_tuning", h, TUNING[k], int(v))
        L.call("mrmf_sector_create", h, int(digit_sum), ctypes.byref(s))
        n = ctypes.c_size_t()
        if L.lib().mrmf_sector_kernel_source(s, dtype, None, 0, ctypes.byref(n)) != 0:
            return None
        buf = ctypes.create_string_buffer(n.value + 1)
        L.call("mrmf_sector_kernel_source", s, dtype, buf, n.value + 1, ctypes.byref(n))
        return buf.value.decode()
    finally:
        if s.value:
            L.lib().mrmf_sector_destroy(s)
        L.lib().mrmf_plan_destroy(h)


def packed_digits(model, digit_sum: int) -> np.ndarray:
    """The packed-digit table the generated sector kernel reads (the sector's states in packed-row order, site
    k's digit in bit_length(d_k - 1) bits, site N - 1 lowest), built from the sector oracle's enumeration."""
    from oracle import sector as osec
    lab = osec.labels(model, digit_sum)
    dims = [s.d for s in model.sites]
    w = [(d - 1).bit_length() for d in dims]
    word = np.dtype(np.uint32 if sum(w) <= 32 else np.uint64)
    digits = np.unravel_index(lab, dims)
    out = np.zeros(lab.size, dtype=np.uint64)
    shift = 0
    for k in range(len(dims) - 1, -1, -1):
        out |= digits[k].astype(np.uint64) << np.uint64(shift)
        shift += w[k]
    return out.astype(word)


def run_sector(model, digit_sum: int, x: np.ndarray, grid: int, tuning=None) -> np.ndarray:
    """y = P H P^T x on the packed sector vector x with the generated sector kernel, emulated on the CPU."""
    f32 = x.dtype == np.complex64
    src = sector_source(model, digit_sum, L.MRMF_DTYPE_C if f32 else L.MRMF_DTYPE_Z, tuning)
    if src is None:
        raise ValueError("the sector does not qualify for the generated kernel")
    lib = _compile(src)
    th = np.ascontiguousarray(model.theta, dtype=np.float32 if f32 else np.float64)
    xx = np.ascontiguousarray(x)
    y = np.full_like(xx, np.nan)
    lab = packed_digits(model, digit_sum)
    rc = lib.emu_run_sector(grid, th.ctypes.data, th.nbytes, xx.ctypes.data, xx.nbytes, y.ctypes.data, y.nbytes,
                            lab.ctypes.data, lab.nbytes)
    if rc != 0:
        raise RuntimeError(f"emu_run_sector failed: {rc}")
    return y


def run_sector_cheb(model, digit_sum: int, x: np.ndarray, prev: np.ndarray, acc: np.ndarray, ea: float, eb: float,
                    eg: float, c: complex, grid: int, tuning=None):
    """The sector kernel with the Chebyshev-step epilogue (c128), emulated on the CPU: returns (prev', acc')
    with prev' = ea P H P^T x + eb x + eg prev and acc' = acc + c prev'."""
    src = sector_source(model, digit_sum, L.MRMF_SOURCE_CHEB, tuning)
    if src is None:
        raise ValueError("the sector does not qualify for the generated kernel")
    lib = _compile(src)
    th = np.ascontiguousarray(model.theta, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.complex128)
    pv = np.array(prev, dtype=np.complex128, copy=True)
    av = np.array(acc, dtype=np.complex128, copy=True)
    lab = packed_digits(model, digit_sum)
    rc = lib.emu_run_sector_cheb(grid, th.ctypes.data, th.nbytes, xx.ctypes.data, xx.nbytes, pv.ctypes.data,
                                 av.ctypes.data, ea, eb, eg, c.real, c.imag, lab.ctypes.data, lab.nbytes)
    if rc != 0:
        raise RuntimeError(f"emu_run_sector_cheb failed: {rc}")
    return pv, av
