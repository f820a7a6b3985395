"""ORACLE (test infrastructure): gradients of the matrix-free map.

For y = H(theta) x with H = sum_p theta_p h_p and an upstream gradient g = dL/dRe y + i dL/dIm y
(PyTorch's convention for real losses of complex tensors):

    dL/dx       = H^dagger g            (here H^dagger is applied with the adjoint term list)
    dL/dtheta_p = Re <g | h_p x>        (h_p x = the oracle matvec with theta = e_p)

and for the Rayleigh quotient L = Re<x|H|x>/<x|x> (Hellmann-Feynman):

    dL/dx = 2 (H x - L x) / <x|x>,   dL/dtheta_p = Re<x|h_p|x> / <x|x>.
"""
from __future__ import annotations

import numpy as np

from . import mf


def apply_h_p(model, x, p: int) -> np.ndarray:
    e = np.zeros(model.n_params)
    e[p] = 1.0
    return mf.matvec(model, x, theta=e)


def adjoint(model, x, g, theta=None):
    theta = model.theta if theta is None else np.asarray(theta, dtype=np.float64)
    gx = mf.matvec(mf.adjoint_model(model), g, theta=theta)
    gt = np.array([np.vdot(g, apply_h_p(model, x, p)).real for p in range(model.n_params)])
    return gx, gt


def rayleigh(model, x):
    x = np.asarray(x, dtype=np.complex128)
    xx = np.vdot(x, x).real
    Hx = mf.matvec(model, x)
    L = np.vdot(x, Hx).real / xx
    gx = 2.0 * (Hx - L * x) / xx
    gt = np.array([np.vdot(x, apply_h_p(model, x, p)).real / xx for p in range(model.n_params)])
    return L, gx, gt
