"""Pins for the restricted-basis oracle (oracle/sector.py, Sec. VI case 2): the worked lookup example of
App. D, sector dimensions from generating functions, the union of sector spectra against the full
spectrum, the one-magnon sector against its closed form, and the membership test against brute force."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import kron
from oracle import sector as S
from workloads.model import OP_LOWER, OP_RAISE, OP_Z, Model, Term, spin_site

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lookup_toy_N4_M0.json")


def test_app_d_lookup_example():
    g = json.load(open(GOLDEN))
    N = g["n_sites"]
    J = 1.7
    # App. D's S_2^+ S_0^- is S_1^+ S_3^- with the sites listed in reverse
    m = Model([spin_site(g["two_s"])] * N, [Term(N - 1 - 2, OP_RAISE, N - 1 - 0, OP_LOWER, 0, 0.5)], np.array([J]))
    Q = g["magnetization"] + N * g["two_s"] // 2
    lab = S.labels(m, Q)
    assert [int(s, 2) for s, _ in g["table"]] == lab.tolist()
    assert [i for _, i in g["table"]] == S.lookup(lab, [int(s, 2) for s, _ in g["table"]]).tolist()
    ex = g["example"]
    assert S.lookup(lab, int(ex["source_label"], 2))[()] == ex["source_index"]
    assert S.lookup(lab, int(ex["invalid_label"], 2))[()] == -1
    H = S.dense(m, Q)
    assert H[ex["target_index"], ex["source_index"]] == ex["coefficient_over_J"] * J   # y[5] += (J/2) x[3]
    # the operator's other update in the sector: |0110> <- |0011> (site 2 raised, site 0 lowered)
    expect = np.zeros((6, 6))
    expect[ex["target_index"], ex["source_index"]] = expect[2, 0] = ex["coefficient_over_J"] * J
    assert np.array_equal(H, expect)


@pytest.mark.parametrize("two_s", [[1] * 8, [2] * 6, [1, 2, 3, 2, 1, 3]])
def test_sector_dimensions_generating_function(two_s):
    """|sector Q| is the z^Q coefficient of prod_i (1 + z + ... + z^{d_i - 1})."""
    m = Model([spin_site(k) for k in two_s], [], np.ones(1))
    poly = np.ones(1, dtype=np.int64)
    for k in two_s:
        poly = np.convolve(poly, np.ones(k + 1, dtype=np.int64))
    for Q in range(len(poly)):
        assert S.labels(m, Q).size == poly[Q]


def test_sector_spectra_make_up_the_full_spectrum():
    """An S_z-conserving Hamiltonian is block diagonal over the sectors: their spectra together are the
    full spectrum (dense Kronecker eigenvalues)."""
    rng = np.random.default_rng(4)
    sites = [spin_site(1), spin_site(2), spin_site(1), spin_site(3)]
    terms = []
    for i, j in ((0, 1), (1, 2), (2, 3), (3, 0), (0, 2)):
        terms += W.xxz_bond_terms(i, j, int(rng.integers(2)), 2)
    terms += [Term(i, OP_Z, -1, OP_Z, 3, float(rng.uniform(-1, 1))) for i in range(4)]
    m = Model(sites, terms, rng.uniform(0.5, 1.5, 4))
    full = np.linalg.eigvalsh(kron.dense_H(m))
    qmax = sum(s.d - 1 for s in sites)
    parts = np.concatenate([np.linalg.eigvalsh(S.dense(m, Q)) for Q in range(qmax + 1)])
    assert np.allclose(np.sort(parts), full, atol=1e-12)


def test_one_magnon_sector_closed_form():
    """Open spin-1/2 XX chain in a field, one up spin (Q = 1): eigenvalues eps_k + h - N h / 2 with
    eps_k = J cos(k pi/(N+1)) (one hopping particle, field energy of one up and N - 1 down spins)."""
    N, J, h = 10, 1.3, 0.25
    m = W.xx_chain_in_field(N, J, h)
    ev = np.linalg.eigvalsh(S.dense(m, 1))
    eps = J * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    assert np.allclose(ev, np.sort(eps + h - N * h / 2), atol=1e-13)


def test_lookup_membership_brute_force():
    rng = np.random.default_rng(9)
    m = Model([spin_site(k) for k in (2, 1, 3, 2, 1)], [], np.ones(1))
    Q = 4
    lab = S.labels(m, Q)
    listed = lab.tolist()
    dims = [s.d for s in m.sites]
    F = rng.integers(0, m.dim, 300)
    got = S.lookup(lab, F)
    for f, r in zip(F.tolist(), got.tolist()):
        digits = np.unravel_index(f, dims)
        if sum(digits) == Q:
            assert r == listed.index(f)
        else:
            assert r == -1


def test_sampled_rows_match_full():
    rng = np.random.default_rng(10)
    m = W.random_model(rng, n_sites=4, max_dim=600, all_channels=False)
    Q = 3
    lab = S.labels(m, Q)
    x = W.random_state(lab.size, rng)
    rows = np.array([0, 3, lab.size - 1])
    assert np.allclose(S.matvec(m, Q, x, rows=rows), S.matvec(m, Q, x)[rows], atol=1e-15, rtol=0)
