"""Pins for the propagation oracle (oracle/propagate.py): closed-form dynamics that do not go through
the matrix exponential (free-fermion magnon hopping, spin rotation, vacuum Rabi oscillation, a
piecewise diagonal drive), unitarity and time reversal."""
import numpy as np
import pytest

import workloads as W
from oracle import propagate as P
from workloads.model import OP_LOWER, OP_RAISE, OP_Z, Model, Term, boson_site, spin_site


@pytest.mark.parametrize("dense", [True, False])
def test_xx_chain_single_magnon(dense):
    """Open spin-1/2 XX chain: one up spin hops with amplitude J/2, so <n|exp(-iHt)|m> =
    sum_k phi_k(n) phi_k(m) exp(-i eps_k t), phi_k(n) = sqrt(2/(N+1)) sin(k n pi/(N+1)),
    eps_k = J cos(k pi/(N+1)) (sites n = 1..N)."""
    N, J, t = 9, 1.3, 2.7
    m = W.xx_chain_in_field(N, J, 0.0)
    start = 3
    x0 = np.zeros(m.dim, dtype=np.complex128)
    x0[2 ** (N - 1 - (start - 1))] = 1.0               # site start - 1 (0-based) up, site 0 most significant
    x = P.propagate(m, x0, t / 3, 3, dense=dense)
    k = np.arange(1, N + 1)
    phi = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(k, k) * np.pi / (N + 1))   # phi[k-1, n-1]
    eps = J * np.cos(k * np.pi / (N + 1))
    amp = (phi * np.exp(-1j * eps * t)[:, None]).T @ phi[:, start - 1]        # amplitude on site n
    expect = np.zeros(m.dim, dtype=np.complex128)
    for n in range(1, N + 1):
        expect[2 ** (N - n)] = amp[n - 1]
    assert np.allclose(x, expect, atol=1e-12, rtol=0)


@pytest.mark.parametrize("two_s", [1, 2, 3])
def test_spin_rotation(two_s):
    """h S_x rotates |m = -s> about x: <S_z>(t) = -s cos(h t) and <S_y>(t) = s sin(h t)."""
    h, t = 0.8, 1.9
    m = Model([spin_site(two_s)], [Term(0, OP_RAISE, -1, OP_Z, 0, 0.5), Term(0, OP_LOWER, -1, OP_Z, 0, 0.5)],
              np.array([h]))
    x0 = np.zeros(two_s + 1, dtype=np.complex128)
    x0[0] = 1.0
    x = P.propagate(m, x0, t, 1)
    s = two_s / 2
    mz = np.arange(two_s + 1) - s
    assert abs(np.vdot(x, mz * x).real - (-s * np.cos(h * t))) <= 1e-13
    # S_y = (S_+ - S_-) / (2i); <S_+> = sum_m c_{m+1}^* C_+(m) c_m
    cp = np.sqrt(s * (s + 1) - mz[:-1] * (mz[:-1] + 1))
    sp = np.sum(np.conj(x[1:]) * cp * x[:-1])
    assert abs(((sp - np.conj(sp)) / 2j).real - s * np.sin(h * t)) <= 1e-13


def test_vacuum_rabi():
    """Resonant Jaynes-Cummings: |up, 0> oscillates with |down, 1>: P_up(t) = cos^2(g t)."""
    w, g = 1.0, 0.37
    m = Model([spin_site(1), boson_site(4)],
              [Term(0, OP_Z, -1, OP_Z, 0, 1.0), Term(1, OP_Z, -1, OP_Z, 0, 1.0),
               Term(0, OP_RAISE, 1, OP_LOWER, 1, 1.0), Term(0, OP_LOWER, 1, OP_RAISE, 1, 1.0)], np.array([w, g]))
    x0 = np.zeros(m.dim, dtype=np.complex128)
    x0[1 * 5 + 0] = 1.0                                  # spin digit 1 (up), boson digit 0
    for t in (0.3, 1.1, 2.5):
        x = P.propagate(m, x0, t, 1)
        assert abs(abs(x[5]) ** 2 - np.cos(g * t) ** 2) <= 1e-13
        assert abs(abs(x[1]) ** 2 - np.sin(g * t) ** 2) <= 1e-13


def test_piecewise_diagonal_drive():
    """H_s = h_s S_z on two spins: commuting steps, so every amplitude picks up exp(-i M dt sum_s h_s)."""
    m = Model([spin_site(2), spin_site(1)], [Term(0, OP_Z, -1, OP_Z, 0, 1.0), Term(1, OP_Z, -1, OP_Z, 0, 1.0)],
              np.array([1.0]))
    hs = np.cos(0.7 * np.arange(6))
    x0 = W.random_state(m.dim, np.random.default_rng(2))
    x = P.propagate(m, x0, 0.25, 6, thetas=[[h] for h in hs])
    mtot = (np.arange(3)[:, None] - 1.0 + np.arange(2)[None, :] - 0.5).ravel()
    assert np.allclose(x, x0 * np.exp(-1j * mtot * 0.25 * hs.sum()), atol=1e-14, rtol=0)


def test_unitarity_and_time_reversal():
    rng = np.random.default_rng(6)
    m = W.random_model(rng, n_sites=4, max_dim=400)
    x0 = W.random_state(m.dim, rng)
    x = P.propagate(m, x0, 0.4, 3)
    assert abs(np.linalg.norm(x) - 1.0) <= 1e-13
    back = P.propagate(m, x, -0.4, 3, dense=False)
    assert np.allclose(back, x0, atol=1e-12, rtol=0)
