"""ORACLE (test infrastructure): Python side of the plain row-by-row evaluation in ``mf_ref.c``.

y = H x is computed one target row at a time as the row of the Kronecker sum that defines H (Sec. I,
with the mixed-radix flattening of Sec. III): every term contributes the products of its local matrix
elements times the entries of x whose digits differ from the row's only on the term's own sites.  The
term list is passed as it is (sites, operator codes, complex coefficients theta[p] w); the built-in local
matrices are built inside the C code from their closed forms, and a general one-site operator is handed
over as the dense matrix of its band.
"""
from __future__ import annotations

import ctypes

import numpy as np

from workloads.model import OP_LOCAL_BASE, OP_LOWER, OP_LOWER2, OP_RAISE, OP_RAISE2, OP_Z, OP_Z2, Model

from . import build as _build

_lib = None
_GENERAL = 16          # operator code of general matrix 0 in mf_ref.c


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.mf_ref_apply.restype = ctypes.c_int
        L.mf_ref_apply.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p, f64p, ctypes.c_int32, i64p,
                                   f64p, ctypes.c_int64, f64p, f64p, ctypes.c_int64, i64p]
        L.mf_ref_threads.restype = ctypes.c_int
        L.mf_ref_threads.argtypes = [ctypes.c_int32]
        L.mf_ref_sources.restype = ctypes.c_int
        L.mf_ref_sources.argtypes = [ctypes.c_int32, i32p, ctypes.c_int32, i32p, ctypes.c_int64,
                                     ctypes.c_int64, i64p]
        _lib = L
    return _lib


def threads(n: int = 0) -> int:
    """Threads of the row loops (OpenMP): n > 0 sets them; returns the count in use."""
    return int(lib().mf_ref_threads(int(n)))


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def term_inputs(model: Model, theta=None):
    """The term list as mf_ref_apply takes it: (term [n, 4] = site_a, op_a, site_b, op_b; coef [n] complex;
    gen_off [g]; gen_mat), built-in operators keeping their codes and every general one-site operator
    replaced by the index of its dense matrix (code 16 + g)."""
    from . import kron
    theta = model.theta if theta is None else np.asarray(theta, dtype=np.float64)
    gen_index: dict = {}
    mats = []
    off = []
    size = 0

    def code(op, site):
        nonlocal size
        if op < OP_LOCAL_BASE:
            return op
        key = (op, site)
        if key not in gen_index:
            Mx = np.ascontiguousarray(kron.general_op(model, op, site), dtype=np.float64)
            gen_index[key] = len(mats)
            mats.append(Mx.ravel())
            off.append(size)
            size += Mx.size
        return _GENERAL + gen_index[key]

    term = np.zeros((len(model.terms), 4), dtype=np.int32)
    coef = np.zeros(len(model.terms), dtype=np.complex128)
    for i, t in enumerate(model.terms):
        if t.site_b >= 0 and t.site_b == t.site_a:
            raise ValueError("a two-site term needs two different sites")
        term[i] = (t.site_a, code(t.op_a, t.site_a), t.site_b, code(t.op_b, t.site_b) if t.site_b >= 0 else 0)
        coef[i] = theta[t.param] * complex(t.w)
    gen_off = np.array(off, dtype=np.int64) if off else np.zeros(1, dtype=np.int64)
    gen_mat = np.concatenate(mats) if mats else np.zeros(1)
    return term, coef, len(mats), gen_off, gen_mat


def matvec(model: Model, x: np.ndarray, theta=None, rows=None) -> np.ndarray:
    """y = H(theta) x in FP64 (x is upcast exactly).  rows: optional int64 target indices; then the
    result holds y at those rows only."""
    kind, twok = model.site_arrays()
    D = model.dim
    xx = np.ascontiguousarray(np.asarray(x).reshape(-1), dtype=np.complex128)
    if xx.shape[0] != D:
        raise ValueError(f"x has {xx.shape[0]} entries, the basis has {D}")
    term, coef, n_gen, gen_off, gen_mat = term_inputs(model, theta)
    if rows is None:
        nrows, rp = D, None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        if rows.size and (rows.min() < 0 or rows.max() >= D):
            raise ValueError("row index out of range")
        nrows, rp = rows.shape[0], _p(rows, ctypes.c_int64)
    y = np.empty(nrows, dtype=np.complex128)
    rc = lib().mf_ref_apply(len(model.sites), _p(kind, ctypes.c_int32), _p(twok, ctypes.c_int32), term.shape[0],
                            _p(term, ctypes.c_int32), _p(coef.view(np.float64), ctypes.c_double), n_gen,
                            _p(gen_off, ctypes.c_int64), _p(gen_mat, ctypes.c_double), D,
                            _p(xx.view(np.float64), ctypes.c_double), _p(y.view(np.float64), ctypes.c_double),
                            nrows, rp)
    if rc != 0:
        raise RuntimeError("mf_ref_apply rejected its input")
    return y


_SHIFT = {OP_Z: 0, OP_Z2: 0, OP_RAISE: 1, OP_LOWER: -1, OP_RAISE2: 2, OP_LOWER2: -2}


def _shift(model: Model, op: int) -> int:
    """Digit shift q of an operator (its matrix elements sit at <n|O|n - q>)."""
    if op >= OP_LOCAL_BASE:
        return int(model.local_ops[op - OP_LOCAL_BASE].shift)
    return _SHIFT[op]


def sources(model: Model, F0: int, count: int) -> np.ndarray:
    """Source index (or -1) of every term for target rows F0..F0+count-1: int64 [count, n_terms]."""
    _, twok = model.site_arrays()
    tt = np.array([(t.site_a, _shift(model, t.op_a), t.site_b, _shift(model, t.op_b) if t.site_b >= 0 else 0)
                   for t in model.terms], dtype=np.int32).reshape(-1, 4)
    out = np.empty((count, len(model.terms)), dtype=np.int64)
    rc = lib().mf_ref_sources(len(model.sites), _p(twok, ctypes.c_int32), len(model.terms),
                              _p(tt, ctypes.c_int32), int(F0), int(count), _p(out, ctypes.c_int64))
    if rc != 0:
        raise RuntimeError("mf_ref_sources rejected its input")
    return out


def adjoint_model(model: Model) -> Model:
    """Term list of H^dagger: every operator replaced by its adjoint, every weight conjugated.  A general
    one-site operator's adjoint is its transposed band (shift -q, <n|O^dag|n + q> = <n + q|O|n>)."""
    from workloads.model import LocalOp, Term
    adj = {OP_Z: OP_Z, OP_Z2: OP_Z2, OP_RAISE: OP_LOWER, OP_LOWER: OP_RAISE, OP_RAISE2: OP_LOWER2,
           OP_LOWER2: OP_RAISE2}
    ops = []
    for lo in model.local_ops:
        d, q = len(lo.values), lo.shift
        ops.append(LocalOp(lo.site, -q, tuple(lo.values[n + q] if 0 <= n + q < d else 0.0 for n in range(d))))

    def a(op):
        return op if op >= OP_LOCAL_BASE else adj[op]     # general op i -> entry i of the adjoint list
    terms = [Term(t.site_a, a(t.op_a), t.site_b, a(t.op_b) if t.site_b >= 0 else t.op_b, t.param,
                  complex(t.w).conjugate()) for t in model.terms]
    return Model(model.sites, terms, model.theta.copy(), name=model.name + "^dag", local_ops=ops)
