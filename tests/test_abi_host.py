"""Host-side tests of the C ABI: the library loads and exports every declared symbol, and the host
plan builder validates input and computes the integer offsets exactly (no GPU needed)."""
import ctypes

import numpy as np
import pytest

import workloads as W
from workloads.model import (OP_LOWER, OP_LOWER2, OP_RAISE, OP_RAISE2, OP_Z, OP_Z2, Model, Term, boson_site,
                             spin_site)
from paper_2606_02169_amd import _lib as L
from tests.helpers import host_plan


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = L.header_symbols()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES)


def test_status_strings():
    for s in range(-6, 1):
        assert L.status_string(s)
    assert L.status_string(L.MRMF_E_NOT_HERMITIAN) == "a parameter group is not Hermitian"


def _offsets(h, n):
    out = (ctypes.c_int64 * max(1, n))()
    L.call("mrmf_plan_offsets", h, out)
    return [out[i] for i in range(n)]


@pytest.mark.parametrize("seed", range(6))
def test_offsets_match_ravel_multi_index(seed):
    """Delta_c of Eq. (sourceoffset) against numpy's C-order flattening of the shifted digits."""
    m = W.random_model(np.random.default_rng(seed), n_sites=5, max_dim=5000)
    st, h = host_plan(m)
    assert st == 0
    n = ctypes.c_int32()
    L.call("mrmf_plan_n_offdiag", h, ctypes.byref(n))
    terms = (ctypes.c_int32 * max(1, n.value))()
    L.call("mrmf_plan_offdiag_terms", h, terms)
    dims = [s.d for s in m.sites]
    shift = {OP_Z: 0, OP_Z2: 0, OP_RAISE: 1, OP_LOWER: -1, OP_RAISE2: 2, OP_LOWER2: -2}
    offs = _offsets(h, n.value)
    expected_terms = [i for i, t in enumerate(m.terms)
                      if shift[t.op_a] != 0 or (t.site_b >= 0 and shift[t.op_b] != 0)]
    assert [terms[i] for i in range(n.value)] == expected_terms
    mid = [d // 2 for d in dims]
    base = np.ravel_multi_index(mid, dims)
    for c, ti in enumerate(expected_terms):
        t = m.terms[ti]
        src = list(mid)
        src[t.site_a] -= shift[t.op_a]
        if t.site_b >= 0:
            src[t.site_b] -= shift[t.op_b]
        src = [min(max(v, 0), d - 1) for v, d in zip(src, dims)]
        # pick a target whose shifted digits are admissible: compare Delta through the flattening
        tgt = list(src)
        tgt[t.site_a] += shift[t.op_a]
        if t.site_b >= 0:
            tgt[t.site_b] += shift[t.op_b]
        if all(0 <= v < d for v, d in zip(tgt, dims)):
            assert np.ravel_multi_index(tgt, dims) - np.ravel_multi_index(src, dims) == offs[c]
    dim = ctypes.c_int64()
    L.call("mrmf_plan_dim", h, ctypes.byref(dim))
    assert dim.value == m.dim
    L.lib().mrmf_plan_destroy(h)


def test_plan_errors():
    ok = Model([spin_site(1), spin_site(2)], W.xxz_bond_terms(0, 1, 0, 0), np.ones(1))
    assert host_plan(ok)[0] == 0
    # same-site pair (a local monomial, not a two-site term)
    bad = Model([spin_site(1), spin_site(2)], [Term(0, OP_RAISE, 0, OP_LOWER, 0, 1.0)], np.ones(1))
    assert host_plan(bad)[0] == L.MRMF_E_INVALID_ARG
    # site out of range, bad op, bad param
    assert host_plan(Model([spin_site(1)], [Term(3, OP_Z)], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
    assert host_plan(Model([spin_site(1)], [Term(0, 7)], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
    assert host_plan(Model([spin_site(1)], [Term(0, OP_Z, -1, OP_Z, 1)], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
    # (S_z)^2 inside a pair term
    assert host_plan(Model([spin_site(2)] * 2, [Term(0, OP_Z2, 1, OP_Z)], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
    # (S_+-)^2 is one-site only
    for op in (OP_RAISE2, OP_LOWER2):
        assert host_plan(Model([spin_site(2)] * 2, [Term(0, op, 1, OP_Z)], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
        assert host_plan(Model([spin_site(2)] * 2, [Term(0, OP_Z, 1, op)], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
    assert host_plan(Model([spin_site(2)], [Term(0, 6)], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
    # trivial site (d = 1) and d > 256
    assert host_plan(Model([spin_site(0)], [], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
    assert host_plan(Model([boson_site(300)], [], np.ones(1)))[0] == L.MRMF_E_INVALID_ARG
    # index overflow: D = 2^62 (single-word index bound)
    assert host_plan(Model([spin_site(1)] * 62, [], np.ones(1)))[0] == L.MRMF_E_OVERFLOW
    assert host_plan(Model([spin_site(1)] * 61, [], np.ones(1)))[0] == 0
    # non-Hermitian group: S_+ without its partner, or J^{+-} != conj(J^{-+})
    nh = Model([spin_site(1)], [Term(0, OP_RAISE, -1, OP_Z, 0, 0.5)], np.ones(1))
    assert host_plan(nh)[0] == L.MRMF_E_NOT_HERMITIAN
    assert host_plan(nh, require_hermitian=False)[0] == 0
    nh2 = Model([spin_site(1)] * 2, [Term(0, OP_RAISE, 1, OP_LOWER, 0, 0.5 + 0.1j),
                                     Term(0, OP_LOWER, 1, OP_RAISE, 0, 0.5 + 0.1j)], np.ones(1))
    assert host_plan(nh2)[0] == L.MRMF_E_NOT_HERMITIAN
    r2 = [Term(0, OP_RAISE2, -1, OP_Z, 0, 0.3 + 0.2j)]
    assert host_plan(Model([spin_site(3)], r2, np.ones(1)))[0] == L.MRMF_E_NOT_HERMITIAN
    assert host_plan(Model([spin_site(3)], r2 + [Term(0, OP_LOWER2, -1, OP_Z, 0, 0.3 - 0.2j)], np.ones(1)))[0] == 0
    h2 = Model([spin_site(1)] * 2, [Term(0, OP_RAISE, 1, OP_LOWER, 0, 0.5 + 0.1j),
                                    Term(1, OP_RAISE, 0, OP_LOWER, 0, 0.5 - 0.1j)], np.ones(1))
    assert host_plan(h2)[0] == 0           # partner written with the sites swapped
    zz = Model([spin_site(1)] * 2, [Term(0, OP_Z, 1, OP_Z, 0, 1j)], np.ones(1))
    assert host_plan(zz)[0] == L.MRMF_E_NOT_HERMITIAN
    # hermiticity is checked per parameter group
    split = Model([spin_site(1)], [Term(0, OP_RAISE, -1, OP_Z, 0, 1.0), Term(0, OP_LOWER, -1, OP_Z, 1, 1.0)],
                  np.ones(2))
    assert host_plan(split)[0] == L.MRMF_E_NOT_HERMITIAN


def test_null_arguments():
    lib = L.lib()
    assert lib.mrmf_plan_create(0, None, 0, None, 0, 0, ctypes.byref(ctypes.c_void_p())) == L.MRMF_E_INVALID_ARG
    assert lib.mrmf_plan_dim(None, None) == L.MRMF_E_INVALID_ARG
    assert lib.mrmf_matvec_z(None, None, None, None, None, None) == L.MRMF_E_INVALID_ARG


def test_named_configs_build():
    for k in (1, 2, 3, 5):
        m, _ = W.config(k, with_state=False)
        st, h = host_plan(m)
        assert st == 0, k
        dim = ctypes.c_int64()
        L.call("mrmf_plan_dim", h, ctypes.byref(dim))
        assert dim.value == m.dim
        L.lib().mrmf_plan_destroy(h)
    assert W.config(2, with_state=False)[0].dim == 2 ** 10 * 3 ** 10
    assert W.config(3, with_state=False)[0].dim == 3 ** 16
    assert W.config(5, with_state=False)[0].dim == 4096 * 65


# ------------------------------------------------------------------ propagation host helpers
@pytest.mark.parametrize("z", [0.0, 1e-6, 0.3, 2.0, 17.5, 140.0, 2500.0])
def test_cheb_bessel_weights(z):
    """The Chebyshev weights J_k(z) of mrmf_propagate_z against scipy.special.jv, and the cut: the
    dropped tail 2 sum_{k > K} |J_k| is at most tol while keeping J_K would exceed it."""
    from scipy.special import jv
    tol, cap = 1e-13, 8192
    out = (ctypes.c_double * cap)()
    n = ctypes.c_int32()
    L.call("mrmf_cheb_bessel", z, tol, cap, out, ctypes.byref(n))
    K = n.value - 1
    got = np.array(out[: n.value])
    ref = jv(np.arange(n.value), z)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.sqrt(z))
    tail = 2 * np.abs(jv(np.arange(K + 1, K + 400), z)).sum()
    assert tail <= tol * 1.0001
    if K > 0:
        assert tail + 2 * abs(ref[K]) > tol
    assert L.lib().mrmf_cheb_bessel(z, tol, max(1, K), None, ctypes.byref(n)) == (
        L.MRMF_E_UNSUPPORTED if K >= 1 else 0)
    assert L.lib().mrmf_cheb_bessel(-1.0, tol, cap, None, ctypes.byref(n)) == L.MRMF_E_INVALID_ARG
    assert L.lib().mrmf_cheb_bessel(z, 0.0, cap, None, ctypes.byref(n)) == L.MRMF_E_INVALID_ARG


def test_norm_bound():
    """mrmf_plan_norm_bound: >= the spectral radius on random models; equal to it for one term."""
    from oracle import kron
    rng = np.random.default_rng(12)
    for _ in range(5):
        m = W.random_model(rng, n_sites=3, max_dim=300)
        st, h = host_plan(m)
        assert st == 0
        b = ctypes.c_double()
        th = np.ascontiguousarray(m.theta, dtype=np.float64)
        L.call("mrmf_plan_norm_bound", h, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(b))
        L.lib().mrmf_plan_destroy(h)
        ev = np.linalg.eigvalsh(kron.dense_H(m))
        assert b.value >= np.max(np.abs(ev)) * (1 - 1e-12)
    one = Model([spin_site(3), boson_site(4)], [Term(1, OP_LOWER, -1, OP_Z, 0, 0.7)], np.array([1.5]))
    st, h = host_plan(one, require_hermitian=False)
    b = ctypes.c_double()
    th = np.array([1.5])
    L.call("mrmf_plan_norm_bound", h, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(b))
    L.lib().mrmf_plan_destroy(h)
    assert abs(b.value - 1.5 * 0.7 * 2.0) <= 1e-15        # ||a|| on n_max = 4 is sqrt(4)


# ------------------------------------------------------------------ restricted basis (host side)
def test_sector_dimensions_and_errors():
    """mrmf_sector_dim against the oracle's enumeration for every digit sum of random lattices; invalid
    digit sums are rejected."""
    from oracle import sector as osec
    rng = np.random.default_rng(21)
    for _ in range(4):
        m = W.random_model(rng, n_sites=5, max_dim=3000)
        st, h = host_plan(m)
        assert st == 0
        qmax = sum(s.d - 1 for s in m.sites)
        for Q in range(qmax + 1):
            sec = ctypes.c_void_p()
            L.call("mrmf_sector_create", h, Q, ctypes.byref(sec))
            n = ctypes.c_int64()
            L.call("mrmf_sector_dim", sec, ctypes.byref(n))
            assert n.value == osec.labels(m, Q).size
            L.lib().mrmf_sector_destroy(sec)
        sec = ctypes.c_void_p()
        assert L.lib().mrmf_sector_create(h, qmax + 1, ctypes.byref(sec)) == L.MRMF_E_INVALID_ARG
        assert L.lib().mrmf_sector_create(h, -1, ctypes.byref(sec)) == L.MRMF_E_INVALID_ARG
        L.lib().mrmf_plan_destroy(h)


# ------------------------------------------------------------------ general one-site operators
def test_general_operator_validation_and_hermiticity():
    from workloads.model import LocalOp
    s1 = spin_site(2)
    up = LocalOp(0, 1, (0.0, 1.2, 0.7))
    dn = W.adjoint_op(up)
    G = W.OP_LOCAL_BASE
    # a Hermitian pair, alone and against a built-in operator on another site
    ok = Model([s1, s1], [Term(0, G, -1, OP_Z, 0, 0.5), Term(0, G + 1, -1, OP_Z, 0, 0.5),
                          Term(0, G, 1, OP_LOWER, 0, 0.3j), Term(0, G + 1, 1, OP_RAISE, 0, -0.3j)], np.ones(1),
               local_ops=[up, dn])
    assert host_plan(ok)[0] == 0
    # the adjoint missing, or with a different table
    lone = Model([s1, s1], [Term(0, G, -1, OP_Z, 0, 0.5)], np.ones(1), local_ops=[up, dn])
    assert host_plan(lone)[0] == L.MRMF_E_NOT_HERMITIAN
    off = LocalOp(0, -1, (1.2, 0.71, 0.0))
    bad = Model([s1], [Term(0, G, -1, OP_Z, 0, 0.5), Term(0, G + 1, -1, OP_Z, 0, 0.5)], np.ones(1),
                local_ops=[up, off])
    assert host_plan(bad)[0] == L.MRMF_E_NOT_HERMITIAN
    # Z S_+ is one band; its adjoint S_- Z written from the other side's matrix product also passes
    z, p, m = W.spin_matrices(2)
    zp, mz = W.band_op(0, z @ p), W.band_op(0, m @ z)
    assert host_plan(Model([s1], [Term(0, G, -1, OP_Z, 0, 1.0), Term(0, G + 1, -1, OP_Z, 0, 1.0)], np.ones(1),
                           local_ops=[zp, mz]))[0] == 0
    # an operator on another site than its term, an index past the list, a shift out of range
    assert host_plan(Model([s1, s1], [Term(1, G, -1, OP_Z)], np.ones(1), local_ops=[up, dn]),
                     require_hermitian=False)[0] == L.MRMF_E_INVALID_ARG
    assert host_plan(Model([s1], [Term(0, G + 2, -1, OP_Z)], np.ones(1), local_ops=[up, dn]),
                     require_hermitian=False)[0] == L.MRMF_E_INVALID_ARG
    assert host_plan(Model([s1], [Term(0, G, -1, OP_Z)], np.ones(1), local_ops=[LocalOp(0, 3, (1.0, 1.0, 1.0))]),
                     require_hermitian=False)[0] == L.MRMF_E_INVALID_ARG
    # channel offsets of general operators: Delta = q_a M_a + q_b M_b
    g = W.random_general_model(np.random.default_rng(4), n_sites=4, max_dim=2000)
    st, h = host_plan(g)
    assert st == 0
    n = ctypes.c_int32()
    L.call("mrmf_plan_n_offdiag", h, ctypes.byref(n))
    terms = (ctypes.c_int32 * max(1, n.value))()
    L.call("mrmf_plan_offdiag_terms", h, terms)
    offs = (ctypes.c_int64 * max(1, n.value))()
    L.call("mrmf_plan_offsets", h, offs)
    M = [int(np.prod([s.d for s in g.sites[k + 1:]])) for k in range(len(g.sites))]
    shift = {OP_Z: 0, OP_Z2: 0, OP_RAISE: 1, OP_LOWER: -1, OP_RAISE2: 2, OP_LOWER2: -2}
    sh = lambda op: g.local_ops[op - W.OP_LOCAL_BASE].shift if op >= W.OP_LOCAL_BASE else shift[op]
    for c in range(n.value):
        t = g.terms[terms[c]]
        want = sh(t.op_a) * M[t.site_a] + (sh(t.op_b) * M[t.site_b] if t.site_b >= 0 else 0)
        assert offs[c] == want
    L.lib().mrmf_plan_destroy(h)


def test_spectral_bounds_argument_checks():
    """mrmf_spectral_bounds rejects bad arguments before any launch: null pointers, a non-Hermitian plan,
    misaligned buffers, too small a scratch (the pointers below are never dereferenced)."""
    import workloads as W
    from workloads.model import OP_RAISE, OP_Z, Model, Term, spin_site
    st, h = host_plan(W.xx_chain_in_field(4, 1.0, 0.2))
    assert st == 0
    try:
        nb = ctypes.c_size_t()
        assert L.lib().mrmf_spectral_bounds_scratch_bytes(h, ctypes.byref(nb)) == 0
        assert nb.value >= 16 and nb.value % 16 == 0
        fake = ctypes.c_void_p(1 << 20)
        fn = L.lib().mrmf_spectral_bounds
        assert fn(None, fake, fake, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(h, None, fake, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(h, fake, fake, fake, None, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(h, ctypes.c_void_p((1 << 20) + 8), fake, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(h, fake, fake, ctypes.c_void_p((1 << 20) + 4), fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(h, fake, fake, fake, fake, nb.value - 16, None) == L.MRMF_E_WORKSPACE
    finally:
        L.lib().mrmf_plan_destroy(h)
    st, q = host_plan(Model([spin_site(1)], [Term(0, OP_RAISE, -1, OP_Z, 0, 1.0)], np.ones(1)),
                      require_hermitian=False)
    assert st == 0
    try:
        fake = ctypes.c_void_p(1 << 20)
        assert L.lib().mrmf_spectral_bounds(q, fake, fake, fake, fake, 1 << 20, None) == L.MRMF_E_NOT_HERMITIAN
    finally:
        L.lib().mrmf_plan_destroy(q)


def test_sector_spectral_bounds_argument_checks():
    """mrmf_sector_spectral_bounds: a scratch of two doubles per block of the reduction, and refusals before
    any launch for null pointers, a non-Hermitian group, misaligned buffers and too small a scratch (the
    pointers below are never dereferenced)."""
    from workloads.model import OP_LOWER, OP_RAISE, Model, Term, spin_site
    from paper_2606_02169_amd.plan import Sector
    m = W.ferrimagnetic_ring(8)
    st, h = host_plan(m)
    assert st == 0
    sec = ctypes.c_void_p()
    try:
        L.call("mrmf_sector_create", h, Sector.digit_sum_of(m.sites, 0.0), ctypes.byref(sec))
        nb = ctypes.c_size_t()
        assert L.lib().mrmf_sector_spectral_bounds_scratch_bytes(sec, ctypes.byref(nb)) == 0
        assert nb.value >= 16 and nb.value % 16 == 0
        assert L.lib().mrmf_sector_spectral_bounds_scratch_bytes(None, ctypes.byref(nb)) == L.MRMF_E_INVALID_ARG
        fake = ctypes.c_void_p(1 << 20)
        fn = L.lib().mrmf_sector_spectral_bounds
        assert fn(None, fake, fake, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(sec, None, fake, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(sec, fake, None, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(sec, fake, fake, None, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(sec, fake, fake, fake, None, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(sec, ctypes.c_void_p((1 << 20) + 8), fake, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(sec, fake, fake, ctypes.c_void_p((1 << 20) + 4), fake, nb.value, None) == L.MRMF_E_INVALID_ARG
        assert fn(sec, fake, fake, fake, fake, nb.value - 16, None) == L.MRMF_E_WORKSPACE
    finally:
        if sec.value:
            L.lib().mrmf_sector_destroy(sec)
        L.lib().mrmf_plan_destroy(h)
    nh = Model([spin_site(1)] * 3, [Term(0, OP_RAISE, 1, OP_LOWER, 0, 1.0)], np.ones(1))
    st, h = host_plan(nh, require_hermitian=False)
    sec = ctypes.c_void_p()
    try:
        L.call("mrmf_sector_create", h, 1, ctypes.byref(sec))
        fake = ctypes.c_void_p(1 << 20)
        assert L.lib().mrmf_sector_spectral_bounds(sec, fake, fake, fake, fake, 1 << 20,
                                                   None) == L.MRMF_E_NOT_HERMITIAN
    finally:
        if sec.value:
            L.lib().mrmf_sector_destroy(sec)
        L.lib().mrmf_plan_destroy(h)


def test_spectral_bounds_many_argument_checks():
    """mrmf_spectral_bounds_many and mrmf_sector_spectral_bounds_many refuse, before any launch, null
    pointers, count < 1, a negative stride, too small a scratch, and plans the one-pass form does not take
    (more than 8 couplings: MRMF_E_UNSUPPORTED); the pointers below are never dereferenced."""
    from workloads.model import OP_LOWER, OP_RAISE, OP_Z, Model, Term, spin_site
    from paper_2606_02169_amd.plan import Sector
    m = W.ferrimagnetic_ring(8)
    st, h = host_plan(m)
    assert st == 0
    sec = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)
    try:
        L.call("mrmf_sector_create", h, Sector.digit_sum_of(m.sites, 0.0), ctypes.byref(sec))
        for fn, qfn, obj in (("mrmf_spectral_bounds_many", "mrmf_spectral_bounds_scratch_bytes", h),
                             ("mrmf_sector_spectral_bounds_many", "mrmf_sector_spectral_bounds_scratch_bytes", sec)):
            nb = ctypes.c_size_t()
            L.call(qfn, obj, ctypes.byref(nb))
            f = getattr(L.lib(), fn)
            assert f(None, fake, fake, 4, 2, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
            assert f(obj, None, fake, 4, 2, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
            assert f(obj, fake, None, 4, 2, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
            assert f(obj, fake, fake, 4, 2, None, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
            assert f(obj, fake, fake, 4, 0, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
            assert f(obj, fake, fake, -1, 2, fake, fake, nb.value, None) == L.MRMF_E_INVALID_ARG
            assert f(obj, fake, fake, 4, 2, ctypes.c_void_p((1 << 20) + 4), fake, nb.value, None) == L.MRMF_E_INVALID_ARG
            assert f(obj, fake, fake, 4, 2, fake, fake, nb.value - 16, None) == L.MRMF_E_WORKSPACE
    finally:
        if sec.value:
            L.lib().mrmf_sector_destroy(sec)
        L.lib().mrmf_plan_destroy(h)
    # nine couplings: more than the one-pass form holds per row
    terms = [Term(i, OP_RAISE, i + 1, OP_LOWER, i, 0.5) for i in range(9)]
    terms += [Term(i, OP_LOWER, i + 1, OP_RAISE, i, 0.5) for i in range(9)]
    terms += [Term(i, OP_Z, -1, OP_Z, i % 9, 0.1) for i in range(10)]
    st, h = host_plan(Model([spin_site(1)] * 10, terms, np.ones(9)))
    assert st == 0
    try:
        nb = ctypes.c_size_t()
        L.call("mrmf_spectral_bounds_scratch_bytes", h, ctypes.byref(nb))
        assert L.lib().mrmf_spectral_bounds_many(h, fake, fake, 9, 2, fake, fake, nb.value, None) == \
            L.MRMF_E_UNSUPPORTED
    finally:
        L.lib().mrmf_plan_destroy(h)


def test_batch_share_input_rules():
    """mrmf_batch_share_input: accepted for lattices with the same local dimensions (different couplings
    or terms), MRMF_E_UNSUPPORTED for lattices of different dimensions, MRMF_E_INVALID_ARG for a flag other
    than 0 or 1; switching back to separate inputs always works."""
    plans = []
    try:
        for m in (W.ferrimagnetic_ring(6), W.ferrimagnetic_ring(6, jz=0.7), W.ferrimagnetic_ring(8)):
            st, h = host_plan(m)
            assert st == 0
            plans.append(h)
        for idx, want in (([0, 1, 0], 0), ([0, 2], L.MRMF_E_UNSUPPORTED)):
            arr = (ctypes.c_void_p * len(idx))(*[plans[i].value for i in idx])
            b = ctypes.c_void_p()
            L.call("mrmf_batch_create", len(idx), arr, 8, ctypes.byref(b))
            try:
                assert L.lib().mrmf_batch_share_input(b, 1) == want
                assert L.lib().mrmf_batch_share_input(b, 2) == L.MRMF_E_INVALID_ARG
                assert L.lib().mrmf_batch_share_input(b, 0) == 0
            finally:
                L.lib().mrmf_batch_destroy(b)
        assert L.lib().mrmf_batch_share_input(None, 1) == L.MRMF_E_INVALID_ARG
    finally:
        for h in plans:
            L.lib().mrmf_plan_destroy(h)


def test_sweep_combine_argument_checks():
    """mrmf_sweep_combine_c refuses, before any launch, null pointers, K < 1, P outside 1..16, n < 1,
    strides shorter than n, misaligned or overlapping buffers (the pointers are never dereferenced)."""
    g, y, th = (ctypes.c_void_p((1 << 40) + (k << 34)) for k in range(3))
    f = L.lib().mrmf_sweep_combine_c

    def call(theta=th, K=4, P=3, n=100, G=g, gs=128, Y=y, ys=128):
        return f(theta, K, P, n, G, gs, Y, ys, None)

    assert call(theta=None) == L.MRMF_E_INVALID_ARG and call(G=None) == L.MRMF_E_INVALID_ARG
    assert call(Y=None) == L.MRMF_E_INVALID_ARG and call(K=0) == L.MRMF_E_INVALID_ARG
    assert call(P=0) == L.MRMF_E_INVALID_ARG and call(P=17) == L.MRMF_E_INVALID_ARG
    assert call(n=0) == L.MRMF_E_INVALID_ARG and call(gs=99) == L.MRMF_E_INVALID_ARG
    assert call(ys=99) == L.MRMF_E_INVALID_ARG
    assert call(G=ctypes.c_void_p(g.value + 4)) == L.MRMF_E_INVALID_ARG
    assert call(Y=ctypes.c_void_p(g.value + 8 * 200)) == L.MRMF_E_INVALID_ARG      # Y inside G's span


def test_lanczos_refuses_non_hermitian_plans():
    """mrmf_lanczos and mrmf_sector_lanczos return MRMF_E_NOT_HERMITIAN, before any launch, for a plan
    built without MRMF_REQUIRE_HERMITIAN whose parameter group is not Hermitian (S_+ S_- without its
    adjoint); the pointers below are never dereferenced."""
    from workloads.model import OP_LOWER, OP_RAISE, Model, Term, spin_site
    m = Model([spin_site(1)] * 3, [Term(0, OP_RAISE, 1, OP_LOWER, 0, 1.0)], np.ones(1))
    assert host_plan(m)[0] == L.MRMF_E_NOT_HERMITIAN
    st, h = host_plan(m, require_hermitian=False)
    assert st == 0
    sec = ctypes.c_void_p()
    try:
        fake = ctypes.c_void_p(1 << 20)
        args = (fake, fake, None, L.MRMF_PREC_Z, 4, L.MRMF_REORTH_CGS2, fake, fake, fake, fake, fake, fake, fake,
                1 << 20, None)
        assert L.lib().mrmf_lanczos(h, *args) == L.MRMF_E_NOT_HERMITIAN
        L.call("mrmf_sector_create", h, 1, ctypes.byref(sec))
        assert L.lib().mrmf_sector_lanczos(sec, *args) == L.MRMF_E_NOT_HERMITIAN
    finally:
        if sec.value:
            L.lib().mrmf_sector_destroy(sec)
        L.lib().mrmf_plan_destroy(h)


def test_lanczos_counts_and_reorth_arguments():
    """mrmf_lanczos_counts refuses null or misaligned pointers before any HIP call, and the Lanczos entry
    point refuses an unknown reorthogonalisation policy before any launch (partial reorthogonalisation,
    policy 3, is a known one; the pointers below are never dereferenced)."""
    fake = ctypes.c_void_p(1 << 20)
    assert L.lib().mrmf_lanczos_counts(None, fake, None) == L.MRMF_E_INVALID_ARG
    assert L.lib().mrmf_lanczos_counts(fake, None, None) == L.MRMF_E_INVALID_ARG
    assert L.lib().mrmf_lanczos_counts(ctypes.c_void_p((1 << 20) + 8), fake, None) == L.MRMF_E_INVALID_ARG
    assert L.MRMF_REORTH_PARTIAL == 3
    st, h = host_plan(W.config(1, with_state=False)[0])
    assert st == 0
    try:
        args = (fake, fake, None, L.MRMF_PREC_Z, 4, 7, fake, fake, fake, fake, fake, fake, fake, 1 << 30, None)
        assert L.lib().mrmf_lanczos(h, *args) == L.MRMF_E_INVALID_ARG
    finally:
        L.lib().mrmf_plan_destroy(h)


def test_noalloc_adjoint_size_limit():
    """mrmf_adjoint_z_noalloc refuses a plan whose partial sums exceed its static array, before any HIP
    call (the pointers below are never dereferenced)."""
    from workloads.model import OP_Z, Model, Term, spin_site
    n_params = 200                                       # 2048 blocks x 200 x 8 B > 1 MiB
    m = Model([spin_site(1)] * 20, [Term(i, OP_Z, -1, OP_Z, i, 1.0) for i in range(20)], np.ones(n_params))
    st, h = host_plan(m)
    assert st == 0
    try:
        nb = ctypes.c_size_t()
        L.call("mrmf_adjoint_scratch_bytes", h, ctypes.byref(nb))
        assert nb.value > L.MRMF_ADJOINT_NOALLOC_SCRATCH_BYTES
        f = [ctypes.c_void_p(k << 30) for k in range(1, 6)]
        fn = L.lib().mrmf_adjoint_z_noalloc
        assert fn(h, f[0], f[1], f[2], f[3], f[4], f[0], None) == L.MRMF_E_WORKSPACE
        assert fn(h, f[0], f[1], f[2], f[3], f[2], f[0], None) == L.MRMF_E_INVALID_ARG   # grad_x aliases x
        assert fn(None, f[0], f[1], f[2], f[3], f[4], f[0], None) == L.MRMF_E_INVALID_ARG
    finally:
        L.lib().mrmf_plan_destroy(h)


def test_propagate_argument_checks():
    """mrmf_propagate_z and mrmf_sector_propagate_z refuse, before any launch, a group that is not
    Hermitian, a scratch smaller than their size query (three vectors), bounds that are not an interval, a
    tolerance outside (0, 1), misaligned or overlapping vectors (the pointers below are distinct, aligned
    and never dereferenced)."""
    from workloads.model import OP_LOWER, OP_RAISE, Model, Term, spin_site
    ptr = [ctypes.c_void_p((1 << 40) + (k << 34)) for k in range(4)]   # ws, x0, x, scratch
    nh = Model([spin_site(1)] * 3, [Term(0, OP_RAISE, 1, OP_LOWER, 0, 1.0)], np.ones(1))
    st, h = host_plan(nh, require_hermitian=False)
    sec = ctypes.c_void_p()
    try:
        L.call("mrmf_sector_create", h, 1, ctypes.byref(sec))
        for fn, obj in (("mrmf_propagate_z", h), ("mrmf_sector_propagate_z", sec)):
            assert getattr(L.lib(), fn)(obj, ptr[0], ptr[0], 0, 0.1, 2, -1.0, 1.0, 1e-12, ptr[1], ptr[2], ptr[3],
                                        1 << 30, None, None) == L.MRMF_E_NOT_HERMITIAN
    finally:
        if sec.value:
            L.lib().mrmf_sector_destroy(sec)
        L.lib().mrmf_plan_destroy(h)
    m = W.ferrimagnetic_ring(8)
    st, h = host_plan(m)
    assert st == 0
    sec = ctypes.c_void_p()
    try:
        from paper_2606_02169_amd.plan import Sector
        L.call("mrmf_sector_create", h, Sector.digit_sum_of(m.sites, 0.0), ctypes.byref(sec))
        dim = ctypes.c_int64()
        L.call("mrmf_sector_dim", sec, ctypes.byref(dim))
        for fn, qfn, obj, n in (("mrmf_propagate_z", "mrmf_propagate_scratch_bytes", h, m.dim),
                                ("mrmf_sector_propagate_z", "mrmf_sector_propagate_scratch_bytes", sec, dim.value)):
            need = ctypes.c_size_t()
            L.call(qfn, obj, ctypes.byref(need))
            assert need.value == 3 * (n * 16 + 256)
            f = getattr(L.lib(), fn)

            def call(dt=0.1, steps=2, lo=-30.0, hi=30.0, tol=1e-12, x0=ptr[1], x=ptr[2], scratch=ptr[3],
                     nbytes=need.value):
                return f(obj, ptr[0], ptr[0], 0, dt, steps, lo, hi, tol, x0, x, scratch, nbytes, None, None)

            assert call(nbytes=need.value - 1) == L.MRMF_E_WORKSPACE
            assert call(lo=1.0, hi=1.0) == L.MRMF_E_INVALID_ARG
            assert call(tol=0.0) == L.MRMF_E_INVALID_ARG and call(tol=1.0) == L.MRMF_E_INVALID_ARG
            assert call(steps=-1) == L.MRMF_E_INVALID_ARG and call(dt=float("nan")) == L.MRMF_E_INVALID_ARG
            assert call(x0=ctypes.c_void_p(ptr[1].value + 8)) == L.MRMF_E_INVALID_ARG
            assert call(x=ctypes.c_void_p(ptr[1].value + 16)) == L.MRMF_E_INVALID_ARG   # partly overlaps x0
            assert call(scratch=ptr[1]) == L.MRMF_E_INVALID_ARG                          # scratch over x0
    finally:
        if sec.value:
            L.lib().mrmf_sector_destroy(sec)
        L.lib().mrmf_plan_destroy(h)
