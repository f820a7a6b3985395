"""ORACLE (test infrastructure): the restricted basis of a globally constrained sector (Sec. VI, case 2;
App. D) and the matvec restricted to it, in FP64, written from the definitions.

The sector is every product state whose local digits sum to Q (for spins n_i = m_i + s_i, so a fixed
total magnetization M = sum m_i is Q = M + sum s_i; with bosons the digit sum is the excitation number).
Its packed storage order is ascending full-basis index F (site 0 most significant, Sec. III), i.e. the
sorted list of admissible labels; lookup(F) is the position of F in that list or -1 (membership test).

The restricted map is the full map between sector states: y = P H P^T x, where P^T scatters the packed
vector into the full basis and P gathers the sector rows back, so a channel whose source leaves the
sector contributes nothing (the failed lookup of Sec. VI.B).  Only ``tests/``, the package's smoke check
and the benchmark's CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np

from . import mf


def labels(model, Q: int) -> np.ndarray:
    """Sorted full-basis indices of the states with digit sum Q (enumeration of the full basis)."""
    dims = [s.d for s in model.sites]
    total = np.zeros(1, dtype=np.int64)
    for d in dims:                      # digit sums in C order, site 0 slowest (np.ravel_multi_index)
        total = (total[:, None] + np.arange(d, dtype=np.int64)[None, :]).ravel()
    return np.flatnonzero(total == Q).astype(np.int64)


def lookup(lab: np.ndarray, F) -> np.ndarray:
    """Packed position of each full index in F, or -1 when F is not a sector state (binary search)."""
    F = np.asarray(F, dtype=np.int64)
    pos = np.searchsorted(lab, F)
    ok = (pos < lab.size) & (lab[np.minimum(pos, lab.size - 1)] == F)
    return np.where(ok, pos, -1).astype(np.int64)


def matvec(model, Q: int, x: np.ndarray, theta=None, lab: np.ndarray | None = None, rows=None) -> np.ndarray:
    """y = P H P^T x on the packed sector vector x (only the packed rows `rows` when given)."""
    lab = labels(model, Q) if lab is None else lab
    full = np.zeros(model.dim, dtype=np.complex128)
    full[lab] = np.asarray(x, dtype=np.complex128)
    if rows is None:
        return mf.matvec(model, full, theta=theta)[lab]
    return mf.matvec(model, full, theta=theta, rows=lab[np.asarray(rows, dtype=np.int64)])


def dense(model, Q: int, theta=None) -> np.ndarray:
    """The restricted Hamiltonian as a dense matrix (small sectors)."""
    lab = labels(model, Q)
    n = lab.size
    cols = []
    for k in range(n):                  # column k = the restricted map applied to unit vector k
        e = np.zeros(n, dtype=np.complex128)
        e[k] = 1.0
        cols.append(matvec(model, Q, e, theta, lab))
    return np.stack(cols, axis=1) if n else np.zeros((0, 0), dtype=np.complex128)
