"""Pins for the oracle: each check ties the oracle to something other than itself (closed forms,
algebraic invariants, library routines, brute force on tiny inputs)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from workloads.model import (OP_LOWER, OP_LOWER2, OP_RAISE, OP_RAISE2, OP_Z, OP_Z2, Model, Term, boson_site,
                             spin_site)
from oracle import grad, kron, lanczos, mf


def dense_from_mf(model, theta=None):
    D = model.dim
    cols = []
    for k in range(D):
        e = np.zeros(D, dtype=np.complex128)
        e[k] = 1.0
        cols.append(mf.matvec(model, e, theta=theta))
    return np.stack(cols, axis=1)


# ------------------------------------------------------------------ local operator algebra
@pytest.mark.parametrize("two_s", [1, 2, 3, 4, 5])
def test_spin_algebra(two_s):
    o = kron.local_ops(spin_site(two_s))
    z, up, dn = o[OP_Z], o[OP_RAISE], o[OP_LOWER]
    s = two_s / 2
    assert np.allclose(z @ up - up @ z, up, atol=1e-14)              # [S_z, S_+] = S_+
    assert np.allclose(up @ dn - dn @ up, 2 * z, atol=1e-13)         # [S_+, S_-] = 2 S_z
    S2 = z @ z + 0.5 * (up @ dn + dn @ up)                            # S^2 = s(s+1)
    assert np.allclose(S2, s * (s + 1) * np.eye(two_s + 1), atol=1e-13)
    assert np.allclose(o[OP_Z2], z @ z)
    assert np.all(np.diff(np.diag(z)) == 1.0) and z[0, 0] == -s       # n = 0 is m = -s


@pytest.mark.parametrize("nmax", [1, 3, 8])
def test_boson_algebra(nmax):
    o = kron.local_ops(boson_site(nmax))
    a, ad, n = o[OP_LOWER], o[OP_RAISE], o[OP_Z]
    assert np.allclose(ad @ a, n, atol=1e-13)                          # n = a^dag a
    comm = a @ ad - ad @ a                                             # truncated [a, a^dag]
    expect = np.eye(nmax + 1)
    expect[nmax, nmax] = -nmax
    assert np.allclose(comm, expect, atol=1e-12)


# ------------------------------------------------------------------ mixed-radix indexing
def test_sources_match_ravel_multi_index():
    rng = np.random.default_rng(7)
    for _ in range(6):
        m = W.random_model(rng, n_sites=5, max_dim=3000)
        dims = [s.d for s in m.sites]
        D = m.dim
        src = mf.sources(m, 0, D)
        digits = np.array(np.unravel_index(np.arange(D), dims)).T       # C order: site 0 slowest
        shift = {OP_Z: 0, OP_Z2: 0, OP_RAISE: 1, OP_LOWER: -1, OP_RAISE2: 2, OP_LOWER2: -2}
        for t_i, t in enumerate(m.terms):
            nd = digits.copy()
            nd[:, t.site_a] -= shift[t.op_a]
            if t.site_b >= 0:
                nd[:, t.site_b] -= shift[t.op_b]
            ok = np.all((nd >= 0) & (nd < np.array(dims)), axis=1)
            expect = np.full(D, -1, dtype=np.int64)
            expect[ok] = np.ravel_multi_index(nd[ok].T, dims)
            assert np.array_equal(src[:, t_i], expect)


def test_spin_half_xor_rule():
    """For spin-1/2 the S_+^i S_-^j source is F with bits i and j flipped (Sec. III, first case)."""
    N = 6
    m = Model([spin_site(1)] * N, [Term(1, OP_RAISE, 4, OP_LOWER, 0, 1.0)], np.ones(1))
    src = mf.sources(m, 0, 2 ** N)[:, 0]
    for F in range(2 ** N):
        bi, bj = (F >> (N - 1 - 1)) & 1, (F >> (N - 1 - 4)) & 1
        ok = bi == 1 and bj == 0
        assert src[F] == ((F ^ (1 << (N - 2)) ^ (1 << (N - 5))) if ok else -1)


def test_uniform_base_d():
    """Homogeneous spin-s: multipliers are powers d^{N-k} (Sec. III, second case)."""
    N, d = 5, 4
    m = Model([spin_site(d - 1)] * N, [Term(k, OP_RAISE, -1, OP_Z, 0, 1.0) for k in range(N)], np.ones(1))
    src = mf.sources(m, 0, d ** N)
    for F in range(0, d ** N, 7):
        for k in range(N):
            nk = (F // d ** (N - 1 - k)) % d
            assert src[F, k] == (F - d ** (N - 1 - k) if nk > 0 else -1)


# ------------------------------------------------------------------ whole H, tiny systems
@pytest.mark.parametrize("seed", range(8))
def test_mf_matches_kronecker(seed):
    rng = np.random.default_rng(seed)
    m = W.random_model(rng, n_sites=int(rng.integers(2, 6)), max_dim=2000,
                       hermitian=bool(seed % 2 == 0))
    H = kron.dense_H(m)
    x = W.random_state(m.dim, rng)
    y = mf.matvec(m, x)
    assert np.linalg.norm(y - H @ x) <= 1e-14 * max(1.0, np.linalg.norm(H @ x))
    rows = rng.choice(m.dim, size=min(50, m.dim), replace=False)
    assert np.allclose(mf.matvec(m, x, rows=rows), (H @ x)[rows], rtol=0, atol=1e-14)


def test_hermitian_models_are_hermitian():
    rng = np.random.default_rng(11)
    for _ in range(5):
        m = W.random_model(rng, n_sites=4, max_dim=800)
        H = dense_from_mf(m)
        assert np.abs(H - H.conj().T).max() < 1e-14
        for p in range(m.n_params):                    # each parameter group separately
            e = np.zeros(m.n_params); e[p] = 1
            Hp = dense_from_mf(m, e)
            assert np.abs(Hp - Hp.conj().T).max() < 1e-14


def test_config1_against_kronecker():
    m, x = W.config(1)
    H = kron.sparse_H(m)
    y = mf.matvec(m, x)
    assert np.linalg.norm(y - H @ x) / np.linalg.norm(H @ x) < 1e-14


# ------------------------------------------------------------------ closed-form physics
def test_singlet_triplet():
    m = W.heisenberg_chain(2, J=1.7)
    ev = np.linalg.eigvalsh(dense_from_mf(m))
    assert np.allclose(ev, [-0.75 * 1.7, 0.25 * 1.7, 0.25 * 1.7, 0.25 * 1.7], atol=1e-14)


@pytest.mark.parametrize("k1,k2", [(1, 2), (2, 3), (1, 3), (3, 3), (2, 2)])
def test_two_spin_total_spin(k1, k2):
    """J S1.S2 = (J/2)[S(S+1) - s1(s1+1) - s2(s2+1)] with multiplicity 2S+1."""
    J = 0.8
    from workloads.configs import open_xxz_chain
    m = open_xxz_chain([k1, k2], np.array([J]), np.array([J]))
    ev = np.sort(np.linalg.eigvalsh(dense_from_mf(m)))
    s1, s2 = k1 / 2, k2 / 2
    expect = []
    S = abs(s1 - s2)
    while S <= s1 + s2 + 1e-9:
        expect += [0.5 * J * (S * (S + 1) - s1 * (s1 + 1) - s2 * (s2 + 1))] * int(round(2 * S + 1))
        S += 1
    assert np.allclose(ev, np.sort(expect), atol=1e-13)


@pytest.mark.parametrize("two_s", [1, 2, 3])
def test_single_spin_in_field(two_s):
    """h_x S_x + h_y S_y + h_z S_z with h_+ = (h_x - i h_y)/2, h_- = conj(h_+) (Sec. IV.A):
    eigenvalues m |h|."""
    hx, hy, hz = 0.3, -0.7, 0.45
    hp = (hx - 1j * hy) / 2
    m = Model([spin_site(two_s)], [Term(0, OP_Z, -1, OP_Z, 0, hz), Term(0, OP_RAISE, -1, OP_Z, 0, hp),
                                   Term(0, OP_LOWER, -1, OP_Z, 0, np.conj(hp))], np.ones(1))
    ev = np.linalg.eigvalsh(dense_from_mf(m))
    s = two_s / 2
    assert np.allclose(ev, (np.arange(two_s + 1) - s) * np.sqrt(hx * hx + hy * hy + hz * hz), atol=1e-14)


def test_single_ion_anisotropy():
    m = Model([spin_site(2)], [Term(0, OP_Z2, -1, OP_Z, 0, 0.5)], np.ones(1))
    assert np.allclose(np.sort(np.linalg.eigvalsh(dense_from_mf(m))), [0, 0.5, 0.5], atol=1e-15)


# ------------------------------------------------------------------ q = +-2 local monomials (App. B)
@pytest.mark.parametrize("kind,k", [("spin", 2), ("spin", 3), ("spin", 4), ("spin", 5), ("boson", 6)])
def test_double_ladder_matrix_elements(kind, k):
    """(S_+)^2 and (S_-)^2 (a^dag^2, a^2) from the oracle's row loop against the closed-form elements
    <m+2|S_+^2|m> = sqrt((s-m)(s+m+1)(s-m-1)(s+m+2)) and <n+2|a^dag^2|n> = sqrt((n+1)(n+2))."""
    site = spin_site(k) if kind == "spin" else boson_site(k)
    d = k + 1
    expect = np.zeros((d, d))
    for n in range(d - 2):
        if kind == "spin":
            s, m = k / 2, n - k / 2
            expect[n + 2, n] = np.sqrt((s - m) * (s + m + 1) * (s - m - 1) * (s + m + 2))
        else:
            expect[n + 2, n] = np.sqrt((n + 1) * (n + 2))
    up2 = dense_from_mf(Model([site], [Term(0, OP_RAISE2, -1, OP_Z, 0, 1.0)], np.ones(1)))
    dn2 = dense_from_mf(Model([site], [Term(0, OP_LOWER2, -1, OP_Z, 0, 1.0)], np.ones(1)))
    assert np.allclose(up2, expect, atol=1e-14, rtol=0)
    assert np.allclose(dn2, expect.T, atol=1e-14, rtol=0)


def test_zero_field_splitting_spin1():
    """D (S_z^2 - s(s+1)/3) + E (S_x^2 - S_y^2) for s = 1 has eigenvalues -2D/3 and D/3 -+ E."""
    Dz, E = 0.83, 0.21
    ev = np.linalg.eigvalsh(dense_from_mf(W.zero_field_splitting(2, Dz, E))) - 2.0 * Dz / 3.0
    assert np.allclose(ev, np.sort([-2 * Dz / 3, Dz / 3 - E, Dz / 3 + E]), atol=1e-14)


def test_zero_field_splitting_spin32():
    """For s = 3/2 the same Hamiltonian has two Kramers doublets at -+sqrt(D^2 + 3 E^2)."""
    Dz, E = 0.57, 0.13
    ev = np.linalg.eigvalsh(dense_from_mf(W.zero_field_splitting(3, Dz, E))) - 5.0 * Dz / 4.0
    r = np.sqrt(Dz * Dz + 3 * E * E)
    assert np.allclose(ev, [-r, -r, r, r], atol=1e-14)


def test_squeezing_oscillator_spectrum():
    """omega n + (g/2)(a^dag^2 + a^2) is a squeezed oscillator: E_n = sqrt(omega^2 - g^2)(n + 1/2) -
    omega/2 for |g| < omega; with a truncation far above the low states they agree to rounding."""
    w, g, nmax = 1.0, 0.35, 90
    m = Model([boson_site(nmax)], [Term(0, OP_Z, -1, OP_Z, 0, 1.0), Term(0, OP_RAISE2, -1, OP_Z, 1, 0.5),
                                   Term(0, OP_LOWER2, -1, OP_Z, 1, 0.5)], np.array([w, g]))
    ev = np.linalg.eigvalsh(dense_from_mf(m))[:6]
    eps = np.sqrt(w * w - g * g)
    assert np.allclose(ev, eps * (np.arange(6) + 0.5) - w / 2, atol=1e-10, rtol=0)


def test_double_ladder_in_products():
    """The oracle's (S_+)^2 on a site of a several-site lattice equals the Kronecker embedding of the
    square of its S_+ (an operator product, not the row loop's two-coefficient product)."""
    sites = [spin_site(3), boson_site(4), spin_site(2)]
    for site in range(3):
        for op, base in ((OP_RAISE2, OP_RAISE), (OP_LOWER2, OP_LOWER)):
            Hm = dense_from_mf(Model(sites, [Term(site, op, -1, OP_Z, 0, 1.0)], np.ones(1)))
            H1 = kron.dense_H(Model(sites, [Term(site, base, -1, OP_Z, 0, 1.0)], np.ones(1)))
            assert np.allclose(Hm, H1 @ H1, atol=1e-13, rtol=0)


@pytest.mark.parametrize("boson_first", [False, True])
def test_jaynes_cummings_spectrum(boson_first):
    w, w0, g, nmax = 1.0, 1.3, 0.17, 6
    b, s = (0, 1) if boson_first else (1, 0)
    sites = [boson_site(nmax), spin_site(1)] if boson_first else [spin_site(1), boson_site(nmax)]
    terms = [Term(b, OP_Z, -1, OP_Z, 0, 1.0), Term(s, OP_Z, -1, OP_Z, 1, 1.0),
             Term(b, OP_RAISE, s, OP_LOWER, 2, 1.0), Term(b, OP_LOWER, s, OP_RAISE, 2, 1.0)]
    m = Model(sites, terms, np.array([w, w0, g]))
    ev = np.sort(np.linalg.eigvalsh(dense_from_mf(m)))
    expect = [-w0 / 2, w * nmax + w0 / 2]
    for n in range(nmax):
        r = np.sqrt((w0 - w) ** 2 / 4 + g * g * (n + 1))
        expect += [w * (n + 0.5) + r, w * (n + 0.5) - r]
    assert np.allclose(ev, np.sort(expect), atol=1e-13)


def test_sz_and_excitation_conservation():
    m = W.ferrimagnetic_ring(6)
    sz = kron.total_sz(m)
    x = W.random_state(m.dim, np.random.default_rng(3))
    sector = sz == 0.5
    xs = np.where(sector, x, 0)
    y = mf.matvec(m, xs)
    assert np.all(y[~sector] == 0.0)                      # exactly zero outside the start sector
    tc = W.tavis_cummings(3, 4, rng=np.random.default_rng(0))
    exc = kron.total_sz(tc)                              # sum S_z + n_b: conserved by TC
    x = W.random_state(tc.dim, np.random.default_rng(4))
    xs = np.where(exc == 1.5, x, 0)
    assert np.all(mf.matvec(tc, xs)[exc != 1.5] == 0.0)


def test_real_hamiltonian_keeps_real_vectors_real():
    m, _ = W.config(2, reduced=6)
    x = np.random.default_rng(1).standard_normal(m.dim).astype(np.complex128)
    assert np.all(mf.matvec(m, x).imag == 0.0)


def test_xx_chain_free_fermions():
    """Open spin-1/2 XX chain in a field: E0 = sum_{eps_k<0} eps_k - N h / 2,
    eps_k = J cos(k pi/(N+1)) + h (Jordan-Wigner)."""
    N, J, h = 12, 1.0, 0.3
    m = W.xx_chain_in_field(N, J, h)
    eps = J * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)) + h
    e0 = eps[eps < 0].sum() - N * h / 2
    x0 = W.random_state(m.dim, np.random.default_rng(5))
    out = lanczos.lanczos(lambda v: mf.matvec(m, v), x0, 120)
    assert abs(out["theta"] - e0) < 1e-11
    Hs = kron.sparse_H(m)
    ev = spla.eigsh(Hs, k=1, which="SA", tol=1e-13)[0][0]
    assert abs(ev - e0) < 1e-10


# ------------------------------------------------------------------ Lanczos
def test_lanczos_config1_against_eigvalsh():
    m, x = W.config(1)
    H = kron.sparse_H(m).toarray().real
    lam = np.linalg.eigvalsh(H)[0]
    out = lanczos.lanczos(lambda v: mf.matvec(m, v), x, 50)
    assert out["theta"] >= lam - 1e-12                          # variational (interlacing)
    assert abs(out["theta"] - lam) <= out["resid"] + 1e-12      # Weyl bound
    assert abs(out["theta"] - lam) < 1e-9
    assert abs(out["resid_est"] - out["resid"]) < 1e-8
    prev = np.inf
    for k in (10, 20, 30, 40):                                  # theta_m non-increasing in m
        t = lanczos.lanczos(lambda v: H @ v, x, k, explicit_residual=False)["theta"]
        assert t <= prev + 1e-12
        prev = t


def test_lanczos_breakdown_on_eigenvector():
    """Fully polarised state of an XXZ chain in a field is an eigenvector: beta_0 = 0."""
    m = W.ferrimagnetic_ring(6)
    x = np.zeros(m.dim, dtype=np.complex128)
    x[-1] = 1.0                                  # all digits maximal: every spin up
    out = lanczos.lanczos(lambda v: mf.matvec(m, v), x, 10)
    assert out["breakdown"] and out["steps"] == 1
    e = mf.matvec(m, x)[-1].real
    assert abs(out["theta"] - e) < 1e-14


# ------------------------------------------------------------------ gradients
def test_adjoint_against_kronecker_and_fd():
    rng = np.random.default_rng(21)
    m = W.random_model(rng, n_sites=4, max_dim=600)
    x = W.random_state(m.dim, rng)
    g = W.random_state(m.dim, rng)
    gx, gt = grad.adjoint(m, x, g)
    H = kron.dense_H(m)
    assert np.linalg.norm(gx - H.conj().T @ g) < 1e-13
    assert np.linalg.norm(gx - H @ g) < 1e-13                    # Hermitian: H^dag g = H g
    # dL/dtheta for L = Re<g|H(theta) x> by central differences
    for p in range(m.n_params):
        e = np.zeros(m.n_params); e[p] = 1e-3
        lp = np.vdot(g, kron.dense_H(m, m.theta + e) @ x).real
        lm = np.vdot(g, kron.dense_H(m, m.theta - e) @ x).real
        assert abs((lp - lm) / 2e-3 - gt[p]) < 1e-11


def test_rayleigh_gradient_fd():
    tc = W.tavis_cummings(3, 5, rng=np.random.default_rng(2))
    x = W.random_state(tc.dim, np.random.default_rng(3))
    L, gx, gt = grad.rayleigh(tc, x)
    H = kron.dense_H(tc)

    def loss(v, th=None):
        Hm = H if th is None else kron.dense_H(tc, th)
        return np.vdot(v, Hm @ v).real / np.vdot(v, v).real

    assert abs(loss(x) - L) < 1e-14
    h = 1e-5
    for p in range(tc.n_params):
        e = np.zeros(tc.n_params); e[p] = h
        fd = (loss(x, tc.theta + e) - loss(x, tc.theta - e)) / (2 * h)
        assert abs(fd - gt[p]) < 1e-9
    for k in np.random.default_rng(0).choice(tc.dim, 8, replace=False):
        for unit in (1.0, 1j):
            d = np.zeros(tc.dim, dtype=np.complex128); d[k] = h * unit
            fd = (loss(x + d) - loss(x - d)) / (2 * h)
            comp = gx[k].real if unit == 1.0 else gx[k].imag
            assert abs(fd - comp) < 1e-8


# ------------------------------------------------------------------ general one-site operators (App. B)
def test_aklt_chain_ground_energy():
    """S.S + (1/3)(S.S)^2 on a periodic spin-1 ring (AKLT): the valence-bond solid is the unique ground
    state with energy exactly -2/3 per bond; on an open chain it is fourfold degenerate (edge spins)."""
    for N in (4, 6):
        ev = np.linalg.eigvalsh(dense_from_mf(W.bilinear_biquadratic_chain(N, 1 / 3)))
        assert abs(ev[0] + 2 * N / 3) <= 1e-12 and ev[1] - ev[0] > 0.1
    ev = np.linalg.eigvalsh(dense_from_mf(W.bilinear_biquadratic_chain(5, 1 / 3, periodic=False)))
    assert np.allclose(ev[:4], -2 * 4 / 3, atol=1e-12) and ev[4] - ev[0] > 0.1


@pytest.mark.parametrize("beta", [-0.7, 0.25, 1.0])
def test_bilinear_biquadratic_two_sites(beta):
    """Two spin-1: S.S = [S(S+1) - 4] / 2 on total spin S, so the levels are x + beta x^2 for
    x = -2 (S = 0, once), -1 (S = 1, 3 times), 1 (S = 2, 5 times)."""
    m = W.bilinear_biquadratic_chain(2, beta, periodic=False)
    ev = np.linalg.eigvalsh(dense_from_mf(m))
    expect = np.sort([-2 + 4 * beta] + [-1 + beta] * 3 + [1 + beta] * 5)
    assert np.allclose(ev, expect, atol=1e-13)


def test_general_operator_tables_against_products():
    """The monomial tables of the bilinear-biquadratic model are bands of products of the oracle's own
    closed-form spin matrices (oracle.kron.local_ops), and the oracle's row loop with general operators
    equals the Kronecker definition on random general models."""
    m = W.bilinear_biquadratic_chain(3, 0.4)
    o = kron.local_ops(spin_site(2))
    z, p, q = o[OP_Z], o[OP_RAISE], o[OP_LOWER]
    want = [z @ z, z @ p, p @ z, z @ q, q @ z, p @ p, q @ q, p @ q, q @ p]
    for k, M in enumerate(want):
        assert np.allclose(kron.general_op(m, W.OP_LOCAL_BASE + k, 0), M, atol=1e-15, rtol=0)
    # the input generator's spin matrices (the source of every general spin table) for s = 1/2 .. 3
    for two_s in range(1, 7):
        o = kron.local_ops(spin_site(two_s))
        for got, op in zip(W.spin_matrices(two_s), (OP_Z, OP_RAISE, OP_LOWER)):
            assert np.allclose(got, o[op], atol=1e-15, rtol=0), (two_s, op)
    rng = np.random.default_rng(17)
    for _ in range(6):
        g = W.random_general_model(rng, n_sites=4, max_dim=900)
        x = W.random_state(g.dim, rng)
        H = kron.dense_H(g)
        assert np.allclose(H, H.conj().T, atol=1e-14)
        assert np.linalg.norm(mf.matvec(g, x) - H @ x) <= 1e-13 * np.linalg.norm(H @ x)


def test_adjoint_model_with_general_operators():
    """The oracle's adjoint term list (transposed bands for general operators) applies H^dagger of the
    Kronecker definition on non-Hermitian random general models."""
    rng = np.random.default_rng(23)
    for _ in range(4):
        m = W.random_general_model(rng, n_sites=4, max_dim=800, hermitian=False)
        g = W.random_state(m.dim, rng)
        H = kron.dense_H(m)
        assert np.linalg.norm(mf.matvec(mf.adjoint_model(m), g) - H.conj().T @ g) <= 1e-13 * np.linalg.norm(H @ g)


def test_truncated_spin_local_sets():
    """A spin chain whose sites keep only some levels (Sec. VI case 1) through general operators on
    d-level sites is the full Hamiltonian projected onto the kept levels (P H P^T with the product
    projector), and keeping every level gives the full spin back."""
    two_s, N, J, h = 3, 3, 0.9, 0.35

    def model(levels, first):
        ops, terms = [], []
        for i in range(N):
            base = W.OP_LOCAL_BASE + len(ops)
            ops += W.truncated_spin_ops(i, two_s, levels, first)
            terms.append(Term(i, base, -1, OP_Z, 1, 1.0))                       # h S_z
        for i in range(N - 1):
            zi, pi_, mi = (W.OP_LOCAL_BASE + 3 * i + k for k in range(3))
            zj, pj, mj = (W.OP_LOCAL_BASE + 3 * (i + 1) + k for k in range(3))
            terms += [Term(i, pi_, i + 1, mj, 0, 0.5), Term(i, mi, i + 1, pj, 0, 0.5), Term(i, zi, i + 1, zj, 0, 1.0)]
        return Model([W.boson_site(levels - 1)] * N, terms, np.array([J, h]), local_ops=ops)

    full = Model([spin_site(two_s)] * N, [Term(i, OP_Z, -1, OP_Z, 1, 1.0) for i in range(N)]
                 + [t for i in range(N - 1) for t in W.xxz_bond_terms(i, i + 1, 0, 0)], np.array([J, h]))
    Hf = kron.dense_H(full)
    assert np.allclose(dense_from_mf(model(two_s + 1, 0)), Hf, atol=1e-14)
    for levels, first in ((2, 0), (3, 1)):
        keep = np.arange(first, first + levels)
        idx = np.ravel_multi_index(np.meshgrid(*([keep] * N), indexing="ij"), [two_s + 1] * N).ravel()
        assert np.allclose(dense_from_mf(model(levels, first)), Hf[np.ix_(idx, idx)], atol=1e-14)
