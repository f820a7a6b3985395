"""The benchmark and test workloads, with their seeds and draw orders.

Random draws use numpy's PCG64 (``numpy.random.default_rng(seed)``).  Couplings are drawn first, in
bond order, then the state vector (real parts for all D entries, then imaginary parts), normalised to
unit 2-norm.  Every input is generated on the host and handed byte-for-byte to both the GPU path and
the oracle.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .model import (BOSON, OP_LOCAL_BASE, OP_LOWER, OP_LOWER2, OP_RAISE, OP_RAISE2, OP_Z, OP_Z2, SPIN, LocalOp,
                    Model, Site, Term, boson_site, dim_of, spin_site, xxz_bond_terms)


# ---------------------------------------------------------------------------------------------
# state vectors
# ---------------------------------------------------------------------------------------------
def random_state(D: int, rng, dtype=np.complex128, nvec: int = 0) -> np.ndarray:
    """x = (re + i im)/||.||, re and im i.i.d. N(0,1).  nvec > 0 gives a [D, nvec] block whose
    columns are normalised separately (the batched layout)."""
    real = np.float32 if np.dtype(dtype) == np.complex64 else np.float64
    shape = (D, nvec) if nvec else (D,)
    re = rng.standard_normal(shape, dtype=real)
    im = rng.standard_normal(shape, dtype=real)
    x = np.empty(shape, dtype=dtype)
    x.real = re
    x.imag = im
    del re, im
    if nvec:
        nrm = np.sqrt(np.sum(np.abs(x.astype(np.complex128)) ** 2, axis=0))
        x /= nrm.astype(real)
    else:
        nrm = np.sqrt(np.vdot(x, x).real)
        x /= real(nrm)
    return x


# ---------------------------------------------------------------------------------------------
# lattices
# ---------------------------------------------------------------------------------------------
def heisenberg_chain(N: int = 12, J: float = 1.0, periodic: bool = False, two_s: int = 1) -> Model:
    """Spin-s Heisenberg chain, one shared coupling parameter theta[0] = J."""
    sites = [spin_site(two_s)] * N
    nb = N if periodic else N - 1
    terms: List[Term] = []
    for i in range(nb):
        terms += xxz_bond_terms(i, (i + 1) % N, 0, 0)
    return Model(sites, terms, np.array([J], dtype=np.float64), name=f"heisenberg_chain_N{N}")


def ferrimagnetic_ring(N: int = 20, jxy: float = 1.0, jz: float = 1.2, dsi: float = 0.5,
                       hz: float = 0.1) -> Model:
    """Alternating s=1/2 (even sites) and s=1 (odd sites) periodic XXZ ring with single-ion
    anisotropy dsi*(S_z)^2 on the s=1 sites and a uniform field hz*S_z.
    Parameters: theta = [J_xy, J_z, D_si, h_z]."""
    sites = [spin_site(1 if i % 2 == 0 else 2) for i in range(N)]
    terms: List[Term] = []
    for i in range(N):
        terms.append(Term(i, OP_Z, -1, OP_Z, 3, 1.0))
        if i % 2 == 1:
            terms.append(Term(i, OP_Z2, -1, OP_Z, 2, 1.0))
    for i in range(N):
        terms += xxz_bond_terms(i, (i + 1) % N, 0, 1)
    return Model(sites, terms, np.array([jxy, jz, dsi, hz], dtype=np.float64),
                 name=f"ferrimagnetic_ring_N{N}")


def square_lattice_bonds(L: int) -> List[Tuple[int, int]]:
    """Periodic L x L lattice, site s = L*r + c; for s = 0.. the bond to the right, then down."""
    bonds = []
    for s in range(L * L):
        r, c = divmod(s, L)
        bonds.append((s, L * r + (c + 1) % L))
        bonds.append((s, L * ((r + 1) % L) + c))
    return bonds


def square_lattice_spin1(L: int = 4, rng=None, jlo: float = 0.5, jhi: float = 1.5,
                         two_s: int = 2) -> Model:
    """Spin-1 Heisenberg model on the periodic L x L lattice with one coupling parameter per bond,
    J_b ~ U[jlo, jhi] drawn in bond order."""
    bonds = square_lattice_bonds(L)
    J = rng.uniform(jlo, jhi, size=len(bonds)) if rng is not None else np.ones(len(bonds))
    terms: List[Term] = []
    for b, (i, j) in enumerate(bonds):
        terms += xxz_bond_terms(i, j, b, b)
    return Model([spin_site(two_s)] * (L * L), terms, np.asarray(J, dtype=np.float64),
                 name=f"square_spin1_{L}x{L}")


def open_xxz_chain(two_s: List[int], jxy: np.ndarray, jz: np.ndarray) -> Model:
    """Open mixed-spin XXZ chain with per-bond parameters theta = [Jxy_0, Jz_0, Jxy_1, Jz_1, ...]."""
    N = len(two_s)
    terms: List[Term] = []
    theta = np.empty(2 * (N - 1), dtype=np.float64)
    for i in range(N - 1):
        terms += xxz_bond_terms(i, i + 1, 2 * i, 2 * i + 1)
        theta[2 * i] = jxy[i]
        theta[2 * i + 1] = jz[i]
    return Model([spin_site(k) for k in two_s], terms, theta, name=f"mixed_chain_N{N}")


def batched_chains(n_lattices: int, rng, n_lo: int = 8, n_hi: int = 16, dmax: int = 1 << 22
                   ) -> List[Model]:
    """Independent open mixed-spin chains: N ~ U{n_lo..n_hi}, 2s ~ U{1,2,3} per site, a lattice with
    D > dmax is redrawn; then (J_xy, J_z) ~ U[-1, 1] per bond."""
    out = []
    for _ in range(n_lattices):
        while True:
            N = int(rng.integers(n_lo, n_hi + 1))
            tk = rng.integers(1, 4, size=N)
            if int(np.prod(tk + 1)) <= dmax:
                break
        J = rng.uniform(-1.0, 1.0, size=(N - 1, 2))
        out.append(open_xxz_chain([int(v) for v in tk], J[:, 0], J[:, 1]))
    return out


def tavis_cummings(n_spins: int = 12, n_max: int = 64, omega: float = 1.0, omega0: float = 1.0,
                   rng=None, glo: float = 0.05, ghi: float = 0.2, jlo: float = -0.1,
                   jhi: float = 0.1) -> Model:
    """n_spins spin-1/2 sites (sites 0..n_spins-1) and one boson mode as the last site:
    H = omega a^dag a + omega0 sum S_z + sum g_i (a S_+ + a^dag S_-) + sum_i J_i S_z^i S_z^{i+1}.
    Parameters: theta = [omega, omega0, g_0.., J_0..]."""
    g = rng.uniform(glo, ghi, size=n_spins) if rng is not None else np.full(n_spins, 0.1)
    J = rng.uniform(jlo, jhi, size=n_spins - 1) if rng is not None else np.zeros(n_spins - 1)
    b = n_spins
    sites = [spin_site(1)] * n_spins + [boson_site(n_max)]
    terms = [Term(b, OP_Z, -1, OP_Z, 0, 1.0)]
    for i in range(n_spins):
        terms.append(Term(i, OP_Z, -1, OP_Z, 1, 1.0))
    for i in range(n_spins):
        p = 2 + i
        terms.append(Term(b, OP_LOWER, i, OP_RAISE, p, 1.0))
        terms.append(Term(b, OP_RAISE, i, OP_LOWER, p, 1.0))
    for i in range(n_spins - 1):
        terms.append(Term(i, OP_Z, i + 1, OP_Z, 2 + n_spins + i, 1.0))
    theta = np.concatenate([[omega, omega0], g, J]).astype(np.float64)
    return Model(sites, terms, theta, name=f"tavis_cummings_{n_spins}x{n_max}")


def staggered_xxz_ring(two_s: List[int], jxy: float = 1.0, jz: float = 1.0, h: float = 0.2,
                       name: str = "staggered_xxz_ring") -> Model:
    """Periodic XXZ chain with sites 2s = two_s[i] and a staggered field +h on even sites, -h on odd sites.
    Parameters: theta = [J_xy, J_z, h] (the sign of the field is carried by the term weight)."""
    N = len(two_s)
    terms: List[Term] = []
    for i in range(N):
        terms.append(Term(i, OP_Z, -1, OP_Z, 2, 1.0 if i % 2 == 0 else -1.0))
    for i in range(N):
        terms += xxz_bond_terms(i, (i + 1) % N, 0, 1)
    return Model([spin_site(k) for k in two_s], terms, np.array([jxy, jz, h], dtype=np.float64), name=name)


def paper_c1() -> Model:
    """The paper's first testbed: spin-1 periodic chain, N = 15, J_xy = J_z = 1, staggered field 0.2."""
    return staggered_xxz_ring([2] * 15, name="spin1_ring_N15")


def paper_c2() -> Model:
    """The paper's second testbed: periodic chain of 6 spin-1/2, then 6 spin-1, then 6 spin-3/2 sites,
    J_xy = J_z = 1, staggered field 0.2 (D = 24^6)."""
    return staggered_xxz_ring([1] * 6 + [2] * 6 + [3] * 6, name="mixed_ring_N18")


def zero_field_splitting(two_s: int, Dz: float, E: float) -> Model:
    """One spin with the zero-field splitting of App. B without its constant:
    Dz (S_z)^2 + (E/2) ((S_+)^2 + (S_-)^2)  =  Dz (S_z)^2 + E ((S_x)^2 - (S_y)^2).  theta = [Dz, E]."""
    terms = [Term(0, OP_Z2, -1, OP_Z, 0, 1.0), Term(0, OP_RAISE2, -1, OP_Z, 1, 0.5),
             Term(0, OP_LOWER2, -1, OP_Z, 1, 0.5)]
    return Model([spin_site(two_s)], terms, np.array([Dz, E], dtype=np.float64), name=f"zfs_2s{two_s}")


def spin_matrices(two_s: int):
    """S_z, S_+, S_- of one spin as dense matrices (basis m = -s .. s, the digit order of Sec. III).

    Used only to write the value tables of general one-site operators, which are inputs handed alike to
    the library and to the oracle; the built-in RAISE / LOWER operators never read them (the library and
    the oracle each evaluate their own ladder elements).  The tables are checked against the oracle's
    local operators and through the AKLT chain's exact ground energy."""
    s = two_s / 2.0
    m = np.arange(two_s + 1) - s
    up = np.zeros((two_s + 1, two_s + 1))
    for i in range(two_s):
        up[i + 1, i] = np.sqrt(s * (s + 1) - m[i] * (m[i] + 1))
    return np.diag(m), up, up.T.copy()


def band_op(site: int, M: np.ndarray) -> LocalOp:
    """The single band of a one-site matrix M as a general operator (raises if M has two bands)."""
    d = M.shape[0]
    shifts = {i - j for i in range(d) for j in range(d) if M[i, j] != 0.0}
    if len(shifts) > 1:
        raise ValueError("operator has more than one band")
    q = shifts.pop() if shifts else 0
    return LocalOp(site, q, tuple(float(M[n, n - q]) if 0 <= n - q < d else 0.0 for n in range(d)))


def bilinear_biquadratic_chain(N: int, beta: float, periodic: bool = True, two_s: int = 2) -> Model:
    """sum over bonds of S_i . S_j + beta (S_i . S_j)^2 (App. B higher powers): the square expands into
    products of one-site monomials S_z^2, S_z S_+, S_+ S_z, S_z S_-, S_- S_z, S_+^2, S_-^2, S_+ S_-, S_- S_+
    on each site, given as general one-site operators.  beta = 1/3 on spin 1 is the AKLT chain.
    theta = [1 (bilinear), beta]."""
    z, p, m = spin_matrices(two_s)
    prods = {"zz": z @ z, "zp": z @ p, "pz": p @ z, "zm": z @ m, "mz": m @ z, "pp": p @ p, "mm": m @ m,
             "pm": p @ m, "mp": m @ p}
    ops, idx = [], {}
    for site in range(N):
        for key, M in prods.items():
            idx[(site, key)] = OP_LOCAL_BASE + len(ops)
            ops.append(band_op(site, M))
    # (S_i . S_j)^2 with S_i . S_j = A + (B + C)/2, A = z z, B = + -, C = - +
    square = [("zz", "zz", 1.0), ("zp", "zm", 0.5), ("pz", "mz", 0.5), ("zm", "zp", 0.5), ("mz", "pz", 0.5),
              ("pp", "mm", 0.25), ("pm", "mp", 0.25), ("mp", "pm", 0.25), ("mm", "pp", 0.25)]
    terms: List[Term] = []
    bonds = [(i, i + 1) for i in range(N - 1)] + ([(N - 1, 0)] if periodic else [])
    for i, j in bonds:
        terms += xxz_bond_terms(i, j, 0, 0)
        for ka, kb, w in square:
            terms.append(Term(i, idx[(i, ka)], j, idx[(j, kb)], 1, w))
    return Model([spin_site(two_s)] * N, terms, np.array([1.0, beta]), name=f"blbq_N{N}",
                 local_ops=ops)


def truncated_spin_ops(site: int, two_s: int, levels: int, first: int = 0) -> List[LocalOp]:
    """S_z, S_+, S_- of a spin s restricted to `levels` consecutive levels m = -s + first .. (a reduced
    local set, Sec. VI case 1: the site is declared with d = levels, e.g. boson_site(levels - 1), and only
    these general operators act on it)."""
    z, p, m = spin_matrices(two_s)
    sl = slice(first, first + levels)
    return [band_op(site, z[sl, sl]), band_op(site, p[sl, sl]), band_op(site, m[sl, sl])]


def adjoint_op(op: LocalOp) -> LocalOp:
    """O^dagger of a real one-band operator: shift -q, <n|O^dag|n + q> = <n + q|O|n>."""
    d = len(op.values)
    q = op.shift
    return LocalOp(op.site, -q, tuple(float(op.values[n + q]) if 0 <= n + q < d else 0.0 for n in range(d)))


def random_general_model(rng, n_sites: int = 4, max_dim: int = 4096, n_params: int = 3, n_ops: int = 6,
                         n_terms: int = 10, hermitian: bool = True) -> Model:
    """Random mixed spin/boson lattice whose terms use random general one-site operators (random band,
    random real values) alone, paired with each other, or with built-in operators; with hermitian=True
    every term comes with its adjoint (operator adjoints and conjugate weight) in the same group."""
    base = random_model(rng, n_sites=n_sites, max_dim=max_dim, n_params=n_params, n_terms=4,
                        hermitian=hermitian, all_channels=False)
    ops: List[LocalOp] = []
    adj_of = {}
    for _ in range(n_ops):
        site = int(rng.integers(n_sites))
        d = base.sites[site].d
        q = int(rng.integers(-(d - 1), d))
        vals = tuple(float(v) if 0 <= n - q < d else 0.0 for n, v in enumerate(rng.uniform(-1, 1, d)))
        a = LocalOp(site, q, vals)
        ops.append(a)
        ops.append(adjoint_op(a))
        ia, ib = OP_LOCAL_BASE + len(ops) - 2, OP_LOCAL_BASE + len(ops) - 1
        adj_of[ia], adj_of[ib] = ib, ia
    builtin_adj = {OP_Z: OP_Z, OP_RAISE: OP_LOWER, OP_LOWER: OP_RAISE}
    terms = list(base.terms)
    for _ in range(n_terms):
        g = OP_LOCAL_BASE + 2 * int(rng.integers(n_ops))
        site = ops[g - OP_LOCAL_BASE].site
        w = complex(rng.uniform(-1, 1), rng.uniform(-1, 1))
        p = int(rng.integers(n_params))
        kind = rng.integers(3)
        if kind == 0 or n_sites == 1:                                   # one-site
            t = Term(site, g, -1, OP_Z, p, w)
            ta = Term(site, adj_of[g], -1, OP_Z, p, w.conjugate())
        else:
            other = [k for k in range(n_sites) if k != site]
            j = int(rng.choice(other))
            if kind == 1:                                               # with a built-in operator
                ob = int(rng.choice([OP_Z, OP_RAISE, OP_LOWER]))
                t = Term(site, g, j, ob, p, w)
                ta = Term(site, adj_of[g], j, builtin_adj[ob], p, w.conjugate())
            else:                                                       # two general operators
                cand = [OP_LOCAL_BASE + 2 * k for k in range(n_ops) if ops[2 * k].site == j]
                if not cand:
                    continue
                h = int(rng.choice(cand))
                t = Term(site, g, j, h, p, w)
                ta = Term(site, adj_of[g], j, adj_of[h], p, w.conjugate())
        terms.append(t)
        if hermitian:
            terms.append(ta)
    return Model(base.sites, terms, base.theta, name="random_general", local_ops=ops)


def xx_chain_in_field(N: int, J: float, h: float) -> Model:
    """Open spin-1/2 XX chain J(S^x S^x + S^y S^y) in a uniform field h S_z: free fermions."""
    terms: List[Term] = [Term(i, OP_Z, -1, OP_Z, 1, 1.0) for i in range(N)]
    for i in range(N - 1):
        terms += [Term(i, OP_RAISE, i + 1, OP_LOWER, 0, 0.5), Term(i, OP_LOWER, i + 1, OP_RAISE, 0, 0.5)]
    return Model([spin_site(1)] * N, terms, np.array([J, h], dtype=np.float64), name=f"xx_chain_N{N}")


_ADJ = {OP_Z: OP_Z, OP_Z2: OP_Z2, OP_RAISE: OP_LOWER, OP_LOWER: OP_RAISE, OP_RAISE2: OP_LOWER2,
        OP_LOWER2: OP_RAISE2}


def random_model(rng, n_sites: int = 4, max_dim: int = 4096, n_params: int = 3, n_terms: int = 12,
                 bosons: bool = True, hermitian: bool = True, all_channels: bool = True) -> Model:
    """Random small mixed spin/boson model with complex weights.  With hermitian=True every term is
    accompanied by its adjoint in the same parameter group, so each h_p is Hermitian.  With
    all_channels=True all nine (alpha, beta) pair channels appear."""
    while True:
        sites = []
        for _ in range(n_sites):
            if bosons and rng.random() < 0.25:
                sites.append(boson_site(int(rng.integers(1, 5))))
            else:
                sites.append(spin_site(int(rng.integers(1, 4))))
        if dim_of(sites) <= max_dim:
            break
    ops2 = [OP_Z, OP_RAISE, OP_LOWER]
    terms: List[Term] = []

    def add(t: Term):
        terms.append(t)
        self_adjoint = (t.op_a in (OP_Z, OP_Z2)) and (t.site_b < 0 or t.op_b == OP_Z)
        if hermitian and not self_adjoint:
            ob = _ADJ[t.op_b] if t.site_b >= 0 else t.op_b
            terms.append(Term(t.site_a, _ADJ[t.op_a], t.site_b, ob, t.param, complex(t.w).conjugate()))

    def weight(self_adjoint: bool):
        re = float(rng.uniform(-1, 1))
        return complex(re, 0.0) if (self_adjoint and hermitian) else complex(re, float(rng.uniform(-1, 1)))

    channels = [(a, b) for a in ops2 for b in ops2] if (all_channels and n_sites > 1) else []
    for (oa, ob) in channels:
        i, j = rng.choice(n_sites, size=2, replace=False)
        sa = (oa == OP_Z and ob == OP_Z)
        add(Term(int(i), oa, int(j), ob, int(rng.integers(n_params)), weight(sa)))
    for _ in range(n_terms):
        if n_sites == 1 or rng.random() < 0.4:
            i = int(rng.integers(n_sites))
            op = int(rng.choice([OP_Z, OP_Z2, OP_RAISE, OP_LOWER, OP_RAISE2, OP_LOWER2]))
            add(Term(i, op, -1, OP_Z, int(rng.integers(n_params)), weight(op in (OP_Z, OP_Z2))))
        else:
            i, j = rng.choice(n_sites, size=2, replace=False)
            oa, ob = int(rng.choice(ops2)), int(rng.choice(ops2))
            add(Term(int(i), oa, int(j), ob, int(rng.integers(n_params)),
                     weight(oa == OP_Z and ob == OP_Z)))
    theta = rng.uniform(0.5, 1.5, size=n_params)
    return Model(sites, terms, theta, name="random")


# ---------------------------------------------------------------------------------------------
# the five named workloads
# ---------------------------------------------------------------------------------------------
def config(k: int, *, reduced: int = 0, with_state: bool = True):
    """Workload k (1..5) with its seed k.  ``reduced`` > 0 shrinks the lattice for oracle-sized runs
    of the same structure: config 2 -> ring of that many sites, config 3 -> L x L lattice with that L,
    config 4 -> that many lattices with N <= 10.  Returns (model or list of models, state)."""
    rng = np.random.default_rng(k)
    if k == 1:
        m = heisenberg_chain(12, 1.0, periodic=False)
        return m, (random_state(m.dim, rng) if with_state else None)
    if k == 2:
        m = ferrimagnetic_ring(reduced or 20)
        return m, (random_state(m.dim, rng) if with_state else None)
    if k == 3:
        m = square_lattice_spin1(reduced or 4, rng)
        return m, (random_state(m.dim, rng, np.complex64) if with_state else None)
    if k == 4:
        if reduced:
            ms = batched_chains(reduced, rng, n_lo=4, n_hi=10, dmax=1 << 14)
        else:
            ms = batched_chains(256, rng)
        xs = [random_state(m.dim, rng, np.complex64, nvec=8) for m in ms] if with_state else None
        return ms, xs
    if k == 5:
        m = tavis_cummings(12, 64, 1.0, 1.0, rng)
        return m, (random_state(m.dim, rng) if with_state else None)
    raise ValueError(k)
