"""ORACLE (test infrastructure): H from its plain definition as a sum of Kronecker products.

    H(theta) = sum_t theta[p_t] w_t  (1 x .. x O_a x .. x O_b x .. x 1)

with site 0 the leftmost factor, so that the flattened index is the mixed-radix integer of Sec. III
(Eq. encode, site 0 most significant; the same as C-order flattening).  Local basis index n = m + s
(notation guide), n = 0 is m = -s; for a boson site n is the occupation (App. C).

Local matrices (Sec. IV.A for spins; standard truncated boson ladder for App. C):
  spin : S_z = diag(m), <m+1|S_+|m> = sqrt(s(s+1) - m(m+1)), S_- = S_+^T, (S_z)^2, (S_+)^2, (S_-)^2
         (the (S_+-)^2 matrices as matrix products of the one-step ones)
  boson: n = diag(n), <n+1|a^dagger|n> = sqrt(n+1), a = (a^dagger)^T, n^2
Only for small systems (dense: D <= a few thousand; sparse: D up to ~1e6).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from workloads.model import (BOSON, OP_LOCAL_BASE, OP_LOWER, OP_LOWER2, OP_RAISE, OP_RAISE2, OP_Z, OP_Z2, SPIN,
                             Model, Site)


def local_ops(site: Site) -> dict:
    d = site.k + 1
    n = np.arange(d, dtype=np.float64)
    if site.kind == SPIN:
        s = site.k / 2.0
        m = n - s
        z = np.diag(m)
        up = np.zeros((d, d))
        for i in range(d - 1):  # <m+1|S_+|m>
            up[i + 1, i] = np.sqrt(s * (s + 1) - m[i] * (m[i] + 1))
    elif site.kind == BOSON:
        z = np.diag(n)
        up = np.zeros((d, d))
        for i in range(d - 1):  # <n+1|a^dag|n>
            up[i + 1, i] = np.sqrt(n[i] + 1)
    else:
        raise ValueError(site.kind)
    return {OP_Z: z, OP_Z2: z @ z, OP_RAISE: up, OP_LOWER: up.T.copy(), OP_RAISE2: up @ up,
            OP_LOWER2: up.T @ up.T}


def general_op(model: Model, op: int, site: int) -> np.ndarray:
    """The d x d matrix of general one-site operator op (App. B local monomials given as one band):
    M[n, n - shift] = values[n] wherever n - shift is a digit."""
    lo = model.local_ops[op - OP_LOCAL_BASE]
    if lo.site != site:
        raise ValueError("a general operator acts on its own site only")
    d = model.sites[site].d
    M = np.zeros((d, d))
    for n in range(d):
        if 0 <= n - lo.shift < d:
            M[n, n - lo.shift] = lo.values[n]
    return M


def op_matrix(model: Model, op: int, site: int) -> np.ndarray:
    if op >= OP_LOCAL_BASE:
        return general_op(model, op, site)
    return local_ops(model.sites[site])[op]


def _factors(model: Model, t):
    facs = [None] * len(model.sites)
    facs[t.site_a] = op_matrix(model, t.op_a, t.site_a)
    if t.site_b >= 0:
        if t.site_b == t.site_a:
            raise ValueError("a two-site term needs two different sites")
        facs[t.site_b] = op_matrix(model, t.op_b, t.site_b)
    return facs


def dense_H(model: Model, theta=None) -> np.ndarray:
    theta = model.theta if theta is None else np.asarray(theta, dtype=np.float64)
    D = model.dim
    H = np.zeros((D, D), dtype=np.complex128)
    for t in model.terms:
        facs = _factors(model, t)
        M = np.ones((1, 1), dtype=np.complex128)
        for i, s in enumerate(model.sites):
            f = facs[i] if facs[i] is not None else np.eye(s.d)
            M = np.kron(M, f)
        H += theta[t.param] * complex(t.w) * M
    return H


def sparse_H(model: Model, theta=None) -> sp.csr_matrix:
    theta = model.theta if theta is None else np.asarray(theta, dtype=np.float64)
    D = model.dim
    H = sp.csr_matrix((D, D), dtype=np.complex128)
    for t in model.terms:
        facs = _factors(model, t)
        M = sp.identity(1, dtype=np.complex128, format="csr")
        for i, s in enumerate(model.sites):
            f = sp.csr_matrix(facs[i]) if facs[i] is not None else sp.identity(s.d, format="csr")
            M = sp.kron(M, f, format="csr")
        H = H + (theta[t.param] * complex(t.w)) * M
    return H.tocsr()


def total_sz(model: Model) -> np.ndarray:
    """Diagonal of sum_i S_z^(i) over spin sites (boson sites contribute their occupation)."""
    d = np.zeros(1)
    for s in model.sites:
        z = np.diag(local_ops(s)[OP_Z])
        d = (d[:, None] + z[None, :]).ravel()
    return d
