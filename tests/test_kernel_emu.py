"""The plan-specialized kernel source, compiled for the CPU against a small HIP emulation layer and run
on host threads: results against the oracle (c128 1e-12, c64 2e-5 relative) and every unmasked buffer
access checked to lie inside x or y.  This covers the kernel generator's indexing on the CPU, for many
tilings, before any of it runs on a GPU."""
import numpy as np
import pytest

import workloads as W
from oracle import mf
from paper_2606_02169_amd import _lib as L
from tests import kernel_emu as E
from tests.helpers import rel_err

TOL_Z, TOL_C = 1e-12, 2e-5


def check(m, x, blocks=None, **kw):
    """Emulated kernel against the oracle: every row, or (blocks = (b0, b1)) the rows of those blocks."""
    y = E.run(m, x, blocks=blocks, **kw)
    ref = mf.matvec(m, x.astype(np.complex128))
    tol = TOL_C if x.dtype == np.complex64 else TOL_Z
    if blocks is not None:
        done = ~np.isnan(y.real)
        assert done.any()
        y, ref = y[done], ref[done]
    err = rel_err(y, ref)
    assert np.all(np.isfinite(y))
    assert err <= tol, err


@pytest.mark.parametrize("k", [1, 5])
def test_small_configs(k):
    m, x = W.config(k)
    blocks = None if k == 1 else (0, 2)       # config 5 (D = 266,240): the rows of the first two blocks
    check(m, x, blocks=blocks)
    check(m, x.astype(np.complex64), blocks=blocks)


def test_ring_reduced():
    m, x = W.config(2, reduced=12)           # D = 6^6
    check(m, x)
    for unrolled in (0, 1, 2):
        check(m, x, unrolled=unrolled)


def test_square_reduced_c64():
    m, x = W.config(3, reduced=3)            # 3x3 spin-1 torus, D = 3^9
    check(m, x)
    check(m, x.astype(np.complex64), unrolled=1)


@pytest.mark.parametrize("seed", range(10))
def test_random_models(seed):
    rng = np.random.default_rng(7000 + seed)
    herm = seed % 4 != 0
    m = W.random_model(rng, n_sites=int(rng.integers(2, 8)), max_dim=12000, hermitian=herm,
                       n_params=int(rng.integers(1, 5)), n_terms=16)
    x = W.random_state(m.dim, rng)
    ref = mf.matvec(m, x)
    for inner, unrolled in ((0, -1), (1, 0), (2, 1), (1, 2)):
        try:                             # the first 8 blocks of a grid of 64: their super-tiles only
            y = E.run(m, x, inner=inner, unrolled=unrolled, require_hermitian=herm, grid=64, blocks=(0, 8))
        except ValueError:               # this tiling does not fit the plan
            continue
        done = ~np.isnan(y.real)
        assert done.any()
        assert rel_err(y[done], ref[done]) <= TOL_Z
    check(m, x.astype(np.complex64), require_hermitian=herm)


@pytest.mark.parametrize("tuning,grid", [({"schedule": 1}, 8), ({"schedule": 1}, 5), ({"branch_skip": 1}, 8),
                                         ({"branch_skip": 1, "schedule": 1, "load_group": 3}, 16),
                                         ({"variant": 1}, 8), ({"variant": 1, "schedule": 1, "load_group": 5}, 5),
                                         ({"schedule": 2}, 8), ({"variant": 1, "schedule": 2}, 7),
                                         ({"addressing": 1}, 8), ({"addressing": 1, "variant": 1}, 6),
                                         ({"far_loads": 10}, 8), ({"far_loads": 12, "addressing": 1}, 8),
                                         ({"far_loads": 10, "variant": 1}, 8),
                                         ({"far_loads": 12, "variant": 1, "far_dir": 1, "load_group": 3}, 5),
                                         ({"far_loads": 11, "variant": 1, "far_dir": 2, "addressing": 1}, 8),
                                         ({"outer_first": 1}, 8), ({"outer_first": 2, "variant": 1}, 8),
                                         ({"outer_first": 3, "schedule": 1}, 5),
                                         ({"outer_first": 1, "variant": 1, "schedule": 2, "addressing": 1}, 7)])
def test_tuning_variants(tuning, grid):
    m, x = W.config(2, reduced=10)           # D = 6^5: 60 super-tiles of the default shape
    check(m, x, tuning=tuning, grid=grid)
    check(m, x.astype(np.complex64), tuning=tuning, grid=grid, unrolled=1)
    m3, x3 = W.config(3, reduced=3)          # 3x3 torus: the super-tiles of the first two blocks
    check(m3, x3, tuning=tuning, grid=grid, inner=4, unrolled=1, blocks=(0, 2))


@pytest.mark.parametrize("variant,top", [(0, 1), (1, 1), (0, 2), (1, 2)])
def test_unrolled_site0(variant, top):
    """Sites 0..top-1 unrolled with the low sites (copies M_s rows apart, staged together in LDS): the
    reduced ring (its closing bond becomes static), the 3x3 torus and random mixed models, both element
    types."""
    tun = {"unroll_top": top, "variant": variant}
    m, x = W.config(2, reduced=10)
    check(m, x, tuning=tun, grid=8, inner=3, unrolled=0)
    check(m, x.astype(np.complex64), tuning=tun, grid=6, inner=3, unrolled=1)
    m3, x3 = W.config(3, reduced=3)
    check(m3, x3, tuning=tun, grid=8, inner=4, unrolled=0 if top == 2 else 1, blocks=(0, 2))
    rng = np.random.default_rng(950 + 2 * variant + top)
    for _ in range(2):
        mr = W.random_model(rng, n_sites=5, max_dim=3000, n_params=2)
        check(mr, W.random_state(mr.dim, rng), tuning=tun, grid=4, inner=2, unrolled=0)


@pytest.mark.parametrize("seed", range(6))
def test_random_models_list_form(seed):
    """The list form on random mixed spin/boson models, several tilings and chunk sizes (small blocks
    with many channels exercise the multi-pass list construction)."""
    rng = np.random.default_rng(7700 + seed)
    herm = seed % 3 != 0
    m = W.random_model(rng, n_sites=int(rng.integers(2, 8)), max_dim=6000, hermitian=herm,
                       n_params=int(rng.integers(1, 5)), n_terms=40)
    x = W.random_state(m.dim, rng)
    ref = mf.matvec(m, x)
    for inner, unrolled, u in ((0, -1, 0), (1, 0, 3), (2, 1, 1), (1, 2, 7)):
        try:
            # a grid of 64 blocks of which the first 8 are emulated: their super-tiles only
            y = E.run(m, x, inner=inner, unrolled=unrolled, require_hermitian=herm,
                      tuning={"variant": 1, "load_group": u}, grid=64, blocks=(0, 8))
        except ValueError:
            continue
        done = ~np.isnan(y.real)
        assert done.any()
        assert rel_err(y[done], ref[done]) <= TOL_Z
    check(m, x.astype(np.complex64), require_hermitian=herm, tuning={"variant": 1})


@pytest.mark.parametrize("variant", [0, 1])
def test_double_ladder_channels(variant):
    """q = +-2 one-site channels (zero-field splitting, squeezing) on inner, unrolled and uniform sites,
    both forms (a subset of the blocks is emulated)."""
    from workloads.model import OP_LOWER2, OP_RAISE2, OP_Z, OP_Z2, Model, Term, boson_site, spin_site
    sites = [spin_site(3), boson_site(4), spin_site(2), spin_site(3), spin_site(2), boson_site(5)]
    terms = []
    for i in range(len(sites) - 1):
        terms += W.xxz_bond_terms(i, i + 1, 0, 0)
    for i, s in enumerate(sites):
        terms += [Term(i, OP_Z2 if s.kind == 0 else OP_Z, -1, OP_Z, 1, 1.0),
                  Term(i, OP_RAISE2, -1, OP_Z, 2, 0.5 + 0.1j * i), Term(i, OP_LOWER2, -1, OP_Z, 2, 0.5 - 0.1j * i)]
    m = Model(sites, terms, np.array([1.0, 0.4, 0.3]))
    x = W.random_state(m.dim, np.random.default_rng(17))
    ref = mf.matvec(m, x)
    for inner, unrolled in ((1, 1), (2, 1), (3, 0), (2, 2)):
        y = E.run(m, x, inner=inner, unrolled=unrolled, tuning={"variant": variant}, grid=32, blocks=(0, 6))
        done = ~np.isnan(y.real)
        assert done.any()
        assert rel_err(y[done], ref[done]) <= TOL_Z, (inner, unrolled)


@pytest.mark.parametrize("variant,addressing", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_chebyshev_step_epilogue(variant, addressing):
    """The c128 kernel with the fused Chebyshev step: prev' = ea H x + eb x + eg prev, acc' = acc + c prev',
    against the oracle's H x on the emulated blocks."""
    rng = np.random.default_rng(31 + variant)
    m = W.random_model(rng, n_sites=5, max_dim=4000, n_params=2)
    x, prev, acc = (W.random_state(m.dim, rng) for _ in range(3))
    ea, eb, eg, c = 0.37, -0.21, -1.0, 0.3 - 0.8j
    hx = mf.matvec(m, x)
    p2, a2 = E.run_cheb(m, x, prev, acc, ea, eb, eg, c, tuning={"variant": variant, "addressing": addressing})
    want_p = ea * hx + eb * x + eg * prev
    assert rel_err(p2, want_p) <= 1e-12
    assert rel_err(a2, acc + c * want_p) <= 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_general_operators(seed):
    """Random general one-site operators (any band, alone, with built-in operators or paired), both
    forms, several tilings, on the emulated blocks."""
    rng = np.random.default_rng(400 + seed)
    m = W.random_general_model(rng, n_sites=int(rng.integers(3, 7)), max_dim=6000, n_params=2)
    x = W.random_state(m.dim, rng)
    ref = mf.matvec(m, x)
    for inner, unrolled, var in ((0, -1, 0), (1, 1, 0), (2, 0, 1), (1, 2, 1)):
        try:
            y = E.run(m, x, inner=inner, unrolled=unrolled, tuning={"variant": var}, grid=32, blocks=(0, 6))
        except ValueError:
            continue
        done = ~np.isnan(y.real)
        assert done.any()
        assert rel_err(y[done], ref[done]) <= TOL_Z, (inner, unrolled, var)


def test_aklt_chain_emulated():
    m = W.bilinear_biquadratic_chain(7, 1 / 3)
    x = W.random_state(m.dim, np.random.default_rng(5))
    check(m, x, tuning={"variant": 1})
    check(m, x.astype(np.complex64), unrolled=1)


@pytest.mark.parametrize("seed", range(8))
def test_adjoint_kernel(seed):
    """The adjoint kernel generated for the plan: grad_x = H g over every row, and the column sums of its
    per-block partials equal Re <g | h_p x> of the oracle, with grids of one row per thread and of several
    rows per thread (ragged last pass); built-in and general one-site operators, real and complex weights."""
    from oracle import grad as ograd
    rng = np.random.default_rng(7600 + seed)
    if seed % 2 == 0:
        m = W.random_model(rng, n_sites=int(rng.integers(2, 7)), max_dim=3000, n_params=int(rng.integers(1, 6)),
                           n_terms=14)
    else:
        m = W.random_general_model(rng, n_sites=int(rng.integers(2, 6)), max_dim=3000, n_params=4)
    x, g = W.random_state(m.dim, rng), W.random_state(m.dim, rng)
    rgx, ref = ograd.adjoint(m, x, g)
    for grid in ((m.dim + 255) // 256, 2):
        gx, part = E.run_grad(m, x, g, grid)
        assert part.shape == (grid, m.n_params) and np.all(np.isfinite(part))
        assert rel_err(gx, rgx) <= 1e-12
        assert np.max(np.abs(part.sum(0) - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_adjoint_kernel_tavis_cummings():
    """Spins with a large boson (d = 17: factor tables in LDS, decode by reciprocal), 24 channels in two
    gather groups, on the generated adjoint kernel."""
    from oracle import grad as ograd
    rng = np.random.default_rng(7700)
    m = W.tavis_cummings(12, 16, 1.0, 0.9, rng)
    x, g = W.random_state(m.dim, rng), W.random_state(m.dim, rng)
    rgx, ref = ograd.adjoint(m, x, g)
    gx, part = E.run_grad(m, x, g, 3)
    assert rel_err(gx, rgx) <= 1e-12
    assert np.max(np.abs(part.sum(0) - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("seed", range(6))
def test_sector_kernel(seed):
    """The kernel generated for a digit-sum sector against the sector oracle (every packed row): rings
    with a bond between the first and last site (rank change over every site between), random mixed
    spin/boson models with general operators, c128 and c64, one block and several rows per thread."""
    from oracle import sector as osec
    rng = np.random.default_rng(7800 + seed)
    if seed == 0:
        m = W.config(2, reduced=8, with_state=False)[0]
    elif seed == 1:
        m = W.tavis_cummings(6, 9, 1.0, 0.8, rng)
    elif seed % 2 == 0:
        m = W.random_model(rng, n_sites=int(rng.integers(3, 7)), max_dim=5000, n_params=3, n_terms=16)
    else:
        m = W.random_general_model(rng, n_sites=int(rng.integers(3, 6)), max_dim=5000, n_params=3)
    qmax = sum(s.d - 1 for s in m.sites)
    for Q in sorted({qmax // 2, max(0, qmax // 2 - 1), qmax}):
        lab = osec.labels(m, Q)
        if lab.size == 0:
            continue
        x = W.random_state(lab.size, rng)
        ref = osec.matvec(m, Q, x, lab=lab)
        for grid in ((lab.size + 255) // 256, 1, 8):
            y = E.run_sector(m, Q, x, grid)
            assert rel_err(y, ref) <= TOL_Z, (Q, grid)
        # the other two row schedules over the XCDs (8 blocks: one per XCD; 16: two per XCD; 3: no XCD split)
        for sched in (L.MRMF_SCHED_XCD_CHUNK, L.MRMF_SCHED_BLOCK_RUN):
            for grid in (3, 8, 16):
                y = E.run_sector(m, Q, x, grid, tuning={"schedule": sched})
                assert rel_err(y, ref) <= TOL_Z, (Q, sched, grid)
        x32 = x.astype(np.complex64)
        y32 = E.run_sector(m, Q, x32, 2)
        assert rel_err(y32, osec.matvec(m, Q, x32.astype(np.complex128), lab=lab)) <= TOL_C


@pytest.mark.parametrize("case", ["odd_ring", "wide_words"])
def test_sector_kernel_spans_and_words(case):
    """The generated sector kernel's two remaining layouts: a ring of odd length, whose closing bond spans
    an odd number of sites (its rank change ends with a one-site segment), and 11 spin-2 sites, whose
    packed digits take 33 bits (8-byte words)."""
    from oracle import sector as osec
    rng = np.random.default_rng(7900)
    if case == "odd_ring":
        m = W.staggered_xxz_ring([1, 2, 1, 2, 1, 2, 2], jxy=0.8, jz=1.1, h=0.3)
        qs = (4, 5)
    else:
        m = W.staggered_xxz_ring([4] * 11, jxy=0.9, jz=0.7, h=0.2)
        qs = (2, 3)
    for Q in qs:
        lab = osec.labels(m, Q)
        assert E.packed_digits(m, Q).dtype == (np.uint64 if case == "wide_words" else np.uint32)
        x = W.random_state(lab.size, rng)
        ref = osec.matvec(m, Q, x, lab=lab)
        for grid in (1, 8):
            assert rel_err(E.run_sector(m, Q, x, grid), ref) <= TOL_Z, (Q, grid)
        x32 = x.astype(np.complex64)
        y32 = E.run_sector(m, Q, x32, 2)
        assert rel_err(y32, osec.matvec(m, Q, x32.astype(np.complex128), lab=lab)) <= TOL_C


@pytest.mark.parametrize("seed", range(4))
def test_sector_chebyshev_step(seed):
    """The sector kernel with the Chebyshev-step epilogue (time propagation in the sector): prev' = ea
    P H P^T x + eb x + eg prev and acc' = acc + c prev' on every packed row against the sector oracle's
    matvec, for the first step's weights (eg = 0) and a later step's, on rings and random models."""
    from oracle import sector as osec
    rng = np.random.default_rng(7900 + seed)
    if seed == 0:
        m = W.config(2, reduced=8, with_state=False)[0]
    elif seed == 1:
        m = W.tavis_cummings(5, 7, 1.0, 0.8, rng)
    else:
        m = W.random_model(rng, n_sites=int(rng.integers(3, 7)), max_dim=5000, n_params=3, n_terms=16)
    qmax = sum(s.d - 1 for s in m.sites)
    Q = qmax // 2
    lab = osec.labels(m, Q)
    x, prev, acc = (W.random_state(lab.size, rng) for _ in range(3))
    hx = osec.matvec(m, Q, x, lab=lab)
    for ea, eb, eg, c in ((0.3, -0.1, 0.0, 0.7 - 0.2j), (0.6, -0.2, -1.0, -0.1 + 0.4j)):
        for grid in ((lab.size + 255) // 256, 3):
            pv, av = E.run_sector_cheb(m, Q, x, prev, acc, ea, eb, eg, c, grid)
            want_p = ea * hx + eb * x + eg * prev
            assert rel_err(pv, want_p) <= TOL_Z, (ea, eg, grid)
            assert rel_err(av, acc + c * want_p) <= TOL_Z, (ea, eg, grid)
