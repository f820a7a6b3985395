"""ORACLE (test infrastructure): Python side of the plain App-A matvec in ``mf_ref.c``.

The term list of a model is first collapsed into the pseudocode's inputs (App. A): per-site one-site
couplings (h_z, h_+, h_-, plus the (S_z)^2 and (S_+-)^2 couplings of App. B) and a pair list with a 3x3 table
J^{alpha beta}, alpha, beta in (z, +, -), each coupling being theta[p] * w summed over the terms that
land on it.  The C code then runs the pseudocode's row loop over all rows or over sampled rows.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from workloads.model import OP_LOCAL_BASE, OP_LOWER, OP_LOWER2, OP_RAISE, OP_RAISE2, OP_Z, OP_Z2, Model

from . import build as _build

_ALPHA = {OP_Z: 0, OP_RAISE: 1, OP_LOWER: 2}
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.mf_ref_matvec.restype = ctypes.c_int
        L.mf_ref_matvec.argtypes = [ctypes.c_int32, i32p, i32p, f64p, ctypes.c_int32, i32p, i32p,
                                    f64p, ctypes.c_int64, f64p, f64p, ctypes.c_int64, i64p]
        L.mf_ref_general_add.restype = ctypes.c_int
        L.mf_ref_general_add.argtypes = [ctypes.c_int32, i32p, ctypes.c_int32, i32p, i64p, f64p, f64p,
                                         ctypes.c_int64, f64p, f64p, ctypes.c_int64, i64p]
        L.mf_ref_sources.restype = ctypes.c_int
        L.mf_ref_sources.argtypes = [ctypes.c_int32, i32p, ctypes.c_int32, i32p, ctypes.c_int64,
                                     ctypes.c_int64, i64p]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def app_a_inputs(model: Model, theta=None):
    """Collapse the term list into (kind, 2s, onsite[N,6], pair_i, pair_j, J[P,3,3])."""
    theta = model.theta if theta is None else np.asarray(theta, dtype=np.float64)
    N = len(model.sites)
    kind, twok = model.site_arrays()
    onsite = np.zeros((N, 6), dtype=np.complex128)  # h_z, h_zz, h_+, h_-, h_++, h_--
    pairs: dict = {}
    Jlist = []
    for t in model.terms:
        if _is_general(t):
            continue                       # handled by general_inputs / mf_ref_general_add
        c = theta[t.param] * complex(t.w)
        if t.site_b < 0:
            col = {OP_Z: 0, OP_Z2: 1, OP_RAISE: 2, OP_LOWER: 3, OP_RAISE2: 4, OP_LOWER2: 5}[t.op_a]
            onsite[t.site_a, col] += c
            continue
        if t.site_a == t.site_b or t.op_a not in _ALPHA or t.op_b not in _ALPHA:
            raise ValueError("pair terms take two different sites and operators in (z, +, -)")
        key = (t.site_a, t.site_b)
        if key not in pairs:
            pairs[key] = len(Jlist)
            Jlist.append(np.zeros((3, 3), dtype=np.complex128))
        Jlist[pairs[key]][_ALPHA[t.op_a], _ALPHA[t.op_b]] += c
    keys = sorted(pairs, key=lambda k: pairs[k])
    pi = np.array([k[0] for k in keys], dtype=np.int32)
    pj = np.array([k[1] for k in keys], dtype=np.int32)
    J = np.array(Jlist, dtype=np.complex128).reshape(-1, 3, 3) if Jlist else np.zeros((0, 3, 3), np.complex128)
    return kind, twok, onsite, pi, pj, J


def _is_general(t) -> bool:
    return t.op_a >= OP_LOCAL_BASE or (t.site_b >= 0 and t.op_b >= OP_LOCAL_BASE)


def _band(model: Model, op: int, site: int):
    """(shift, table at target digits) of one operator: a general one's given table, or the band of the
    closed-form local matrix of a built-in one (oracle.kron.local_ops)."""
    from . import kron
    if op >= OP_LOCAL_BASE:
        lo = model.local_ops[op - OP_LOCAL_BASE]
        if lo.site != site:
            raise ValueError("a general operator acts on its own site only")
        return lo.shift, np.asarray(lo.values, dtype=np.float64)
    Mx = kron.local_ops(model.sites[site])[op]
    d = Mx.shape[0]
    q = {OP_Z: 0, OP_Z2: 0, OP_RAISE: 1, OP_LOWER: -1, OP_RAISE2: 2, OP_LOWER2: -2}[op]
    return q, np.array([Mx[n, n - q] if 0 <= n - q < d else 0.0 for n in range(d)])


def general_inputs(model: Model, theta=None):
    """Terms with a general one-site operator as (gterm [n,4], toff [n,2], tab, c [n] complex)."""
    theta = model.theta if theta is None else np.asarray(theta, dtype=np.float64)
    gterm, toff, tab, c = [], [], [], []
    size = 0
    for t in model.terms:
        if not _is_general(t):
            continue
        qa, ta = _band(model, t.op_a, t.site_a)
        if t.site_b >= 0:
            qb, tb = _band(model, t.op_b, t.site_b)
        else:
            qb, tb = 0, np.zeros(0)
        gterm.append((t.site_a, qa, t.site_b, qb))
        toff.append((size, size + ta.size))
        tab += [ta, tb]
        size += ta.size + tb.size
        c.append(theta[t.param] * complex(t.w))
    return (np.array(gterm, dtype=np.int32).reshape(-1, 4), np.array(toff, dtype=np.int64).reshape(-1, 2),
            np.concatenate(tab) if tab else np.zeros(1), np.array(c, dtype=np.complex128))


def matvec(model: Model, x: np.ndarray, theta=None, rows=None) -> np.ndarray:
    """y = H(theta) x in FP64 (x is upcast exactly).  rows: optional int64 target indices; then the
    result holds y at those rows only."""
    kind, twok, onsite, pi, pj, J = app_a_inputs(model, theta)
    D = model.dim
    xx = np.ascontiguousarray(np.asarray(x).reshape(-1), dtype=np.complex128)
    if xx.shape[0] != D:
        raise ValueError(f"x has {xx.shape[0]} entries, the basis has {D}")
    onsite = np.ascontiguousarray(onsite)
    J = np.ascontiguousarray(J)
    if rows is None:
        nrows, rp = D, None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        if rows.size and (rows.min() < 0 or rows.max() >= D):
            raise ValueError("row index out of range")
        nrows, rp = rows.shape[0], _p(rows, ctypes.c_int64)
    y = np.empty(nrows, dtype=np.complex128)
    rc = lib().mf_ref_matvec(len(model.sites), _p(kind, ctypes.c_int32), _p(twok, ctypes.c_int32),
                             _p(onsite.view(np.float64), ctypes.c_double), len(pi),
                             _p(pi, ctypes.c_int32), _p(pj, ctypes.c_int32),
                             _p(J.view(np.float64), ctypes.c_double), D,
                             _p(xx.view(np.float64), ctypes.c_double),
                             _p(y.view(np.float64), ctypes.c_double), nrows, rp)
    if rc != 0:
        raise RuntimeError("mf_ref_matvec rejected its input")
    gterm, toff, tab, c = general_inputs(model, theta)
    if gterm.shape[0]:
        rc = lib().mf_ref_general_add(len(model.sites), _p(twok, ctypes.c_int32), gterm.shape[0],
                                      _p(gterm, ctypes.c_int32), _p(toff, ctypes.c_int64),
                                      _p(tab, ctypes.c_double), _p(c.view(np.float64), ctypes.c_double), D,
                                      _p(xx.view(np.float64), ctypes.c_double),
                                      _p(y.view(np.float64), ctypes.c_double), nrows, rp)
        if rc != 0:
            raise RuntimeError("mf_ref_general_add rejected its input")
    return y


def sources(model: Model, F0: int, count: int) -> np.ndarray:
    """Source index (or -1) of every term for target rows F0..F0+count-1: int64 [count, n_terms]."""
    _, twok = model.site_arrays()
    al = {OP_Z: 0, OP_Z2: 0, OP_RAISE: 1, OP_LOWER: 2, OP_RAISE2: 3, OP_LOWER2: 4}
    tt = np.array([(t.site_a, al[t.op_a], t.site_b, al[t.op_b] if t.site_b >= 0 else 0)
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
