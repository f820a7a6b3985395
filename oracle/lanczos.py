"""ORACLE (test infrastructure): plain FP64 Lanczos with full CGS2 reorthogonalisation.

The paper only needs the map x -> H x for a Krylov eigensolver (Sec. I) and specifies none, so this is
the textbook Hermitian Lanczos recurrence, written out step by step:

    v_0 = x / ||x||
    for j = 0 .. m-1:
        w      = H v_j
        alpha_j = Re <v_j | w>
        w     -= alpha_j v_j + beta_{j-1} v_{j-1}
        twice:  c = V^H w ;  w -= V c            (V = [v_0 .. v_j], classical Gram-Schmidt x 2)
        beta_j = ||w||
        stop if beta_j <= 1e-14 * ||T||  (Gershgorin estimate of the tridiagonal matrix so far)
        v_{j+1} = w / beta_j

The lowest Ritz value theta and its vector s come from the k x k tridiagonal T (scipy's
eigh_tridiagonal as the library primitive), u = V s, with the estimate beta_{k-1} |s_{k-1}| and the
explicit residual ||H u - theta u||.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos(matvec, v0: np.ndarray, m: int, reorth: bool = True, tol: float = 1e-14,
            explicit_residual: bool = True) -> dict:
    v = np.asarray(v0, dtype=np.complex128).copy()
    nrm = np.sqrt(np.vdot(v, v).real)
    if nrm == 0.0:
        raise ValueError("zero start vector")
    V = [v / nrm]
    alpha, beta = [], []
    tnorm = 0.0
    breakdown = False
    for j in range(m):
        w = np.asarray(matvec(V[j]), dtype=np.complex128)
        a = float(np.vdot(V[j], w).real)
        w = w - a * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        if reorth:
            Vm = np.stack(V, axis=1)
            for _ in range(2):
                c = Vm.conj().T @ w
                w = w - Vm @ c
        b = float(np.sqrt(np.vdot(w, w).real))
        alpha.append(a)
        beta.append(b)
        tnorm = max(tnorm, abs(a) + b + (beta[j - 1] if j > 0 else 0.0))
        if j == m - 1:
            break
        if b <= tol * tnorm:
            breakdown = True
            break
        V.append(w / b)
    k = len(alpha)
    al = np.array(alpha)
    be = np.array(beta)
    if k == 1:
        theta, s = al[0], np.ones(1)
    else:
        ev, evec = eigh_tridiagonal(al, be[: k - 1], select="i", select_range=(0, 0))
        theta, s = float(ev[0]), evec[:, 0]
    u = np.zeros_like(V[0])
    for i in range(k):
        u += s[i] * V[i]
    out = dict(alpha=al, beta=be, theta=float(theta), ritz_vector=u, steps=k, breakdown=breakdown,
               resid_est=float(be[k - 1] * abs(s[k - 1])))
    if explicit_residual:
        r = np.asarray(matvec(u)) - theta * u
        out["resid"] = float(np.sqrt(np.vdot(r, r).real))
    return out
