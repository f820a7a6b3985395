"""ctypes binding of libmrmf.so: the C ABI declared in include/mrmf.h, one Python function per entry
point with the same name.  Argument marshalling only; all work happens in the HIP library."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrmf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mrmf.h")

MRMF_OK = 0
MRMF_E_INVALID_ARG = -1
MRMF_E_OVERFLOW = -2
MRMF_E_NOT_HERMITIAN = -3
MRMF_E_HIP = -4
MRMF_E_UNSUPPORTED = -5
MRMF_E_WORKSPACE = -6
MRMF_ADJOINT_NOALLOC_SCRATCH_BYTES = 1 << 20
MRMF_SPIN, MRMF_BOSON = 0, 1
MRMF_OP_Z, MRMF_OP_Z2, MRMF_OP_RAISE, MRMF_OP_LOWER, MRMF_OP_RAISE2, MRMF_OP_LOWER2 = 0, 1, 2, 3, 4, 5
MRMF_REQUIRE_HERMITIAN = 1
MRMF_PREC_Z, MRMF_PREC_C_IN_Z = 0, 1
MRMF_REORTH_CGS2, MRMF_REORTH_NONE, MRMF_REORTH_CGS2_COND, MRMF_REORTH_PARTIAL = 0, 1, 2, 3
MRMF_KERNEL_AUTO, MRMF_KERNEL_GENERIC, MRMF_KERNEL_SPECIALIZED = 0, 1, 2
MRMF_DTYPE_Z, MRMF_DTYPE_C = 0, 1
MRMF_TUNE_SCHEDULE, MRMF_TUNE_BRANCH_SKIP, MRMF_TUNE_LOAD_GROUP, MRMF_TUNE_BLOCKS_PER_CU = 0, 1, 2, 3
MRMF_TUNE_VARIANT, MRMF_VARIANT_MASKED, MRMF_VARIANT_LIST = 4, 0, 1
MRMF_TUNE_ADDRESSING = 5
MRMF_TUNE_CHEB_FUSED = 6
MRMF_TUNE_WAVES_PER_EU = 7
MRMF_TUNE_FAR_LOADS = 8
MRMF_TUNE_GRAD_BLOCKS_PER_CU = 9
MRMF_TUNE_OUTER_FIRST = 10
MRMF_TUNE_UNROLL_TOP = 11
MRMF_TUNE_FAR_DIR = 12
MRMF_TUNE_CHEB_MERGE = 13
MRMF_SOURCE_CHEB = 2
MRMF_SOURCE_GRAD = 3
MRMF_BATCH_SCHED_RUNS, MRMF_BATCH_SCHED_WINDOWS, MRMF_BATCH_SCHED_XCD_CHUNK = 0, 1, 2
MRMF_SCHED_WINDOWS, MRMF_SCHED_XCD_CHUNK, MRMF_SCHED_BLOCK_RUN = 0, 1, 2


class mrmf_site(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32)]


class mrmf_term(ctypes.Structure):
    _fields_ = [("site_a", ctypes.c_int32), ("op_a", ctypes.c_int32), ("site_b", ctypes.c_int32),
                ("op_b", ctypes.c_int32), ("param", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("w_re", ctypes.c_double), ("w_im", ctypes.c_double)]


class mrmf_local_op(ctypes.Structure):
    _fields_ = [("site", ctypes.c_int32), ("shift", ctypes.c_int32), ("values", ctypes.POINTER(ctypes.c_double))]


MRMF_OP_LOCAL_BASE = 16


class MrmfError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t
_P = ctypes.POINTER

SIGNATURES = {
    "mrmf_status_string": (ctypes.c_char_p, [_i32]),
    "mrmf_version": (_i32, []),
    "mrmf_plan_create": (_i32, [_i32, _P(mrmf_site), _i32, _P(mrmf_term), _i32, _u32, _P(_vp)]),
    "mrmf_plan_create_ex": (_i32, [_i32, _P(mrmf_site), _i32, _P(mrmf_term), _i32, _u32, _i32, _P(mrmf_local_op),
                                   _P(_vp)]),
    "mrmf_plan_destroy": (None, [_vp]),
    "mrmf_plan_dim": (_i32, [_vp, _P(_i64)]),
    "mrmf_plan_n_offdiag": (_i32, [_vp, _P(_i32)]),
    "mrmf_plan_offdiag_terms": (_i32, [_vp, _P(_i32)]),
    "mrmf_plan_offsets": (_i32, [_vp, _P(_i64)]),
    "mrmf_plan_workspace_bytes": (_i32, [_vp, _P(_sz)]),
    "mrmf_plan_upload": (_i32, [_vp, _vp, _sz, _vp]),
    "mrmf_matvec_z": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mrmf_matvec_c": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mrmf_debug_sources": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp]),
    "mrmf_plan_set_kernel": (_i32, [_vp, _i32, _i32, _i32]),
    "mrmf_plan_prepare": (_i32, [_vp, _i32]),
    "mrmf_plan_set_tuning": (_i32, [_vp, _i32, _i32]),
    "mrmf_plan_autotune": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _P(_i32)]),
    "mrmf_plan_set_shape": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32]),
    "mrmf_plan_kernel_info": (_i32, [_vp, _i32, _P(_i32)]),
    "mrmf_plan_kernel_source": (_i32, [_vp, _i32, ctypes.c_char_p, _sz, _P(_sz)]),
    "mrmf_adjoint_scratch_bytes": (_i32, [_vp, _P(_sz)]),
    "mrmf_adjoint_z": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mrmf_adjoint_z_noalloc": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mrmf_reduce_scratch_bytes": (_i32, [_i64, _P(_sz)]),
    "mrmf_dot_z": (_i32, [_i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mrmf_norm_z": (_i32, [_i64, _vp, _vp, _vp, _sz, _vp]),
    "mrmf_lanczos_scratch_bytes": (_i32, [_vp, _i32, _i32, _P(_sz)]),
    "mrmf_lanczos_counts": (_i32, [_vp, _vp, _vp]),
    "mrmf_lanczos": (_i32, [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            _sz, _vp]),
    "mrmf_propagate_scratch_bytes": (_i32, [_vp, _P(_sz)]),
    "mrmf_propagate_z": (_i32, [_vp, _vp, _vp, _i64, ctypes.c_double, _i32, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, _vp, _vp, _vp, _sz, _P(_i32), _vp]),
    "mrmf_plan_norm_bound": (_i32, [_vp, _P(ctypes.c_double), _P(ctypes.c_double)]),
    "mrmf_spectral_bounds_scratch_bytes": (_i32, [_vp, _P(ctypes.c_size_t)]),
    "mrmf_spectral_bounds": (_i32, [_vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "mrmf_spectral_bounds_many": (_i32, [_vp, _vp, _vp, ctypes.c_int64, _i32, _vp, _vp, ctypes.c_size_t, _vp]),
    "mrmf_cheb_bessel": (_i32, [ctypes.c_double, ctypes.c_double, _i32, _P(ctypes.c_double), _P(_i32)]),
    "mrmf_sector_create": (_i32, [_vp, _i32, _P(_vp)]),
    "mrmf_sector_destroy": (None, [_vp]),
    "mrmf_sector_dim": (_i32, [_vp, _P(_i64)]),
    "mrmf_sector_workspace_bytes": (_i32, [_vp, _P(_sz)]),
    "mrmf_sector_upload": (_i32, [_vp, _vp, _sz, _vp]),
    "mrmf_sector_matvec_z": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mrmf_sector_matvec_c": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mrmf_sector_generated": (_i32, [_vp, _i32, _P(_i32)]),
    "mrmf_sector_kernel_source": (_i32, [_vp, _i32, _vp, _sz, _P(_sz)]),
    "mrmf_sector_labels": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _sz, _vp]),
    "mrmf_sector_lookup": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "mrmf_sector_lanczos_scratch_bytes": (_i32, [_vp, _i32, _i32, _P(_sz)]),
    "mrmf_sector_lanczos": (_i32, [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _sz, _vp]),
    "mrmf_sector_spectral_bounds_scratch_bytes": (_i32, [_vp, _P(_sz)]),
    "mrmf_sector_spectral_bounds": (_i32, [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mrmf_sector_spectral_bounds_many": (_i32, [_vp, _vp, _vp, ctypes.c_int64, _i32, _vp, _vp, _sz, _vp]),
    "mrmf_sector_propagate_scratch_bytes": (_i32, [_vp, _P(_sz)]),
    "mrmf_sector_propagate_z": (_i32, [_vp, _vp, _vp, _i64, ctypes.c_double, _i32, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _vp, _vp, _vp, _sz, _P(_i32), _vp]),
    "mrmf_batch_create": (_i32, [_i32, _P(_vp), _i32, _P(_vp)]),
    "mrmf_batch_destroy": (None, [_vp]),
    "mrmf_batch_total_elems": (_i32, [_vp, _P(_i64)]),
    "mrmf_batch_offsets": (_i32, [_vp, _P(_i64)]),
    "mrmf_batch_theta_offsets": (_i32, [_vp, _P(_i32)]),
    "mrmf_batch_workspace_bytes": (_i32, [_vp, _P(_sz)]),
    "mrmf_batch_upload": (_i32, [_vp, _vp, _sz, _vp]),
    "mrmf_batch_matvec_c": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mrmf_batch_graph_capture": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mrmf_batch_graph_launch": (_i32, [_vp, _vp]),
    "mrmf_batch_autotune": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _P(_i32)]),
    "mrmf_batch_set_shape": (_i32, [_vp, _i32, _i32]),
    "mrmf_batch_set_schedule": (_i32, [_vp, _i32]),
    "mrmf_batch_get_shape": (_i32, [_vp, _P(_i32)]),
    "mrmf_batch_share_input": (_i32, [_vp, _i32]),
    "mrmf_sweep_combine_c": (_i32, [_vp, _i32, _i32, _i64, _vp, _i64, _vp, _i64, _vp]),
}

_lib = None


def header_symbols():
    """Names of every function declared in include/mrmf.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mrmf_[a-z0-9_]+)\s*\(", text)))


def lib():
    """The loaded library.  Raises if libmrmf.so has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2606_02169_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().mrmf_status_string(int(s)).decode()


def check(status: int, where: str):
    if status != MRMF_OK:
        raise MrmfError(status, where)


def call(name: str, *args):
    """Call an entry point and raise MrmfError on a non-OK status."""
    st = getattr(lib(), name)(*args)
    check(st, name)
    return st


def __getattr__(name):
    # mrmf_* names resolve to the raw library functions (same names as the C ABI)
    if name.startswith("mrmf_") and name in SIGNATURES:
        return getattr(lib(), name)
    raise AttributeError(name)
