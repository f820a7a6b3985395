"""ORACLE (test infrastructure): exact time propagation x(t) = exp(-i H t) x0 in FP64.

The paper names exact flat-basis propagation under repeatedly rebuilt or driven Hamiltonians as a use
case of the map x -> H x (Sec. VII, Sec. VIII) without fixing a propagator, so this is the plain
definition: for a piecewise-constant drive theta_0, theta_1, ... held for dt each,

    x_{s+1} = exp(-i dt H(theta_s)) x_s

with H(theta) the Kronecker-sum Hamiltonian of ``kron.sparse_H``.  The exponential is applied by
scipy's ``expm_multiply`` (a library primitive) or, for small D, by the dense ``scipy.linalg.expm``.
Only ``tests/``, the package's smoke check and the benchmark's CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import kron


def propagate(model, x0: np.ndarray, dt: float, n_steps: int = 1, thetas=None, dense: bool | None = None):
    """x after n_steps steps of length dt; thetas = per-step parameter vectors (default: model.theta)."""
    x = np.asarray(x0, dtype=np.complex128).copy()
    if dense is None:
        dense = model.dim <= 2048
    for s in range(n_steps):
        th = model.theta if thetas is None else np.asarray(thetas[s], dtype=np.float64)
        if dense:
            x = sla.expm(-1j * dt * kron.dense_H(model, th)) @ x
        else:
            x = spla.expm_multiply(-1j * dt * kron.sparse_H(model, th).astype(np.complex128), x)
    return x
