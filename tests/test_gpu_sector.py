"""Restricted basis of a fixed digit-sum sector (mrmf_sector_*, Sec. VI case 2) against the restricted-
basis oracle: labels and lookups bit-exact, the sector matvec to the matvec tolerances, the worked lookup
example of App. D, sector Lanczos against closed forms and the oracle, and the 20-site ring's S_z = 0
sector on sampled rows."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import lanczos as olz
from oracle import sector as osec
from tests.helpers import rel_err
from workloads.model import OP_LOWER, OP_RAISE, Model, Term, spin_site

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")
TOL_Z, TOL_C = 1e-12, 2e-5


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def sector(model, Q, kind="auto", **kw):
    from paper_2606_02169_amd.plan import Plan, Sector
    p = Plan.from_model(model, **kw)
    if kind == "generic":
        p.set_kernel("generic")
    return Sector(p, Q)


@pytest.mark.parametrize("kind", ["auto", "generic"])
@pytest.mark.parametrize("seed", range(8))
def test_sector_random_models(seed, kind):
    rng = np.random.default_rng(6100 + seed)
    herm = seed % 3 != 0
    m = W.random_model(rng, n_sites=int(rng.integers(2, 7)), max_dim=20000, hermitian=herm,
                       n_params=int(rng.integers(1, 4)), n_terms=20)
    qmax = sum(s.d - 1 for s in m.sites)
    Q = int(rng.integers(0, qmax + 1))
    lab = osec.labels(m, Q)
    print(f"seed={seed} kind={kind} D={m.dim} Q={Q} Dr={lab.size}", flush=True)
    S = sector(m, Q, kind, require_hermitian=herm)
    assert S.dim == lab.size
    assert S.generated() == S.generated(torch.complex64) == (kind == "auto")
    assert np.array_equal(S.labels().cpu().numpy(), lab)
    F = np.concatenate([lab[:50], rng.integers(-3, m.dim + 3, 400)])
    assert np.array_equal(S.lookup(t(F.astype(np.int64))).cpu().numpy(), osec.lookup(lab, F))
    x = W.random_state(lab.size, rng)
    y = S.matvec(t(m.theta), t(x)).cpu().numpy()
    assert rel_err(y, osec.matvec(m, Q, x, lab=lab)) <= TOL_Z
    x32 = x.astype(np.complex64)
    y32 = S.matvec(t(m.theta.astype(np.float32)), t(x32)).cpu().numpy()
    ref32 = osec.matvec(m, Q, x32.astype(np.complex128), theta=m.theta.astype(np.float32).astype(np.float64), lab=lab)
    assert rel_err(y32, ref32) <= TOL_C


@pytest.mark.parametrize("case", ["odd_ring", "wide_words"])
def test_sector_packed_digit_layouts(case):
    """The generated kernel's packed digits in both word sizes, through the upload and mrmf_sector_labels
    (bit-exact), and its matvec against the oracle: a 7-site mixed ring (closing bond over an odd span,
    4-byte words) and 11 spin-2 sites (33 bits of digits, 8-byte words)."""
    rng = np.random.default_rng(6400)
    if case == "odd_ring":
        m = W.staggered_xxz_ring([1, 2, 1, 2, 1, 2, 2], jxy=0.8, jz=1.1, h=0.3)
        qs = (4, 5)
    else:
        m = W.staggered_xxz_ring([4] * 11, jxy=0.9, jz=0.7, h=0.2)
        qs = (2, 3, 6)
    for Q in qs:
        lab = osec.labels(m, Q)
        S = sector(m, Q)
        print(f"{case} Q={Q} Dr={lab.size}", flush=True)
        assert S.dim == lab.size and S.generated() and S.generated(torch.complex64)
        assert np.array_equal(S.labels().cpu().numpy(), lab)
        x = W.random_state(lab.size, rng)
        y = S.matvec(t(m.theta), t(x)).cpu().numpy()
        assert rel_err(y, osec.matvec(m, Q, x, lab=lab)) <= TOL_Z
        x32 = x.astype(np.complex64)
        y32 = S.matvec(t(m.theta.astype(np.float32)), t(x32)).cpu().numpy()
        ref32 = osec.matvec(m, Q, x32.astype(np.complex128), theta=m.theta.astype(np.float32).astype(np.float64),
                            lab=lab)
        assert rel_err(y32, ref32) <= TOL_C


def test_app_d_lookup_example_on_gpu():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lookup_toy_N4_M0.json")))
    N, J = g["n_sites"], 1.7
    m = Model([spin_site(1)] * N, [Term(N - 1 - 2, OP_RAISE, N - 1 - 0, OP_LOWER, 0, 0.5)], np.array([J]))
    S = sector(m, g["magnetization"] + N // 2, require_hermitian=False)
    assert S.labels().cpu().tolist() == [int(s, 2) for s, _ in g["table"]]
    ex = g["example"]
    F = t(np.array([int(ex["source_label"], 2), int(ex["invalid_label"], 2)], dtype=np.int64))
    assert S.lookup(F).cpu().tolist() == [ex["source_index"], -1]
    x = np.zeros(6, dtype=np.complex128)
    x[ex["source_index"]] = 1.0
    y = S.matvec(t(m.theta), t(x)).cpu().numpy()
    expect = np.zeros(6, dtype=np.complex128)
    expect[ex["target_index"]] = ex["coefficient_over_J"] * J
    assert np.array_equal(y, expect)


def test_one_magnon_sector_lanczos():
    """Sector Lanczos on the open XX chain (N = 24) in its one-magnon (24 states) and two-magnon (276
    states) sectors against the free-fermion ground energies."""
    N, J, h = 24, 1.0, 0.2
    m = W.xx_chain_in_field(N, J, h)
    eps = np.sort(J * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)))
    for Q, e0 in ((1, eps[0] + h - N * h / 2), (2, eps[0] + eps[1] + 2 * h - N * h / 2)):
        S = sector(m, Q)
        x = W.random_state(S.dim, np.random.default_rng(Q))
        r = S.lanczos(t(m.theta), t(x), min(S.dim, 60))["result"].cpu().numpy()
        assert abs(r[0] - e0) <= 1e-12


def test_ring_sector_lanczos_reduced():
    """The 20-site ring's structure at N = 12 in its S_z = 0 sector: sector Lanczos against the oracle's
    Lanczos on the oracle's sector matvec."""
    m, _ = W.config(2, reduced=12)
    Q = Sector_digit_sum(m, 0.0)
    lab = osec.labels(m, Q)
    x = W.random_state(lab.size, np.random.default_rng(5))
    S = sector(m, Q)
    r = S.lanczos(t(m.theta), t(x), 80)["result"].cpu().numpy()
    o = olz.lanczos(lambda v: osec.matvec(m, Q, v, lab=lab), x, 80)
    assert abs(r[0] - o["theta"]) <= 1e-10 * abs(o["theta"])
    # partial reorthogonalisation reaches the same Ritz value with fewer Gram-Schmidt passes
    out = S.lanczos(t(m.theta), t(x), 80, reorth="partial")
    rp, passes = out["result"].cpu().numpy(), int(out["counts"].cpu().numpy()[1])
    print(f"sector Lanczos: cgs2 {r[0]!r} partial {rp[0]!r} ({passes} passes) oracle {o['theta']!r}", flush=True)
    assert abs(rp[0] - o["theta"]) <= 1e-10 * abs(o["theta"])
    assert passes < 40


@pytest.mark.parametrize("reorth", ["cgs2", "partial"])
def test_ring_sector_lanczos_fp32_form(reorth):
    """Sector Lanczos with the c64 sector matvec inside the FP64 recurrence (the 12-site ring's S_z = 0
    sector): the ground energy within 1e-5 of the oracle's FP64 sector Lanczos, and not below it by more
    than FP32 rounding (no spurious level)."""
    m, _ = W.config(2, reduced=12)
    Q = Sector_digit_sum(m, 0.0)
    lab = osec.labels(m, Q)
    x = W.random_state(lab.size, np.random.default_rng(5))
    S = sector(m, Q)
    th = t(m.theta)
    r = S.lanczos(th, t(x), 80, precision="c_in_z", reorth=reorth, theta_c=th.float())["result"].cpu().numpy()
    o = olz.lanczos(lambda v: osec.matvec(m, Q, v, lab=lab), x, 80)
    rel = (r[0] - o["theta"]) / abs(o["theta"])
    print(f"sector fp32 form ({reorth}): {r[0]!r} oracle fp64 {o['theta']!r} rel {rel:.2e}", flush=True)
    assert int(r[3]) == 80
    assert abs(rel) <= 1e-5 and rel >= -1e-6


def Sector_digit_sum(m, M):
    from paper_2606_02169_amd.plan import Sector
    return Sector.digit_sum_of(m.sites, M)


def test_ring20_sz0_sector_sampled():
    """20-site ferrimagnetic ring, S_z = 0 sector (7,873,260 states): sampled rows against the oracle,
    labels of the sampled rows against the oracle's enumeration."""
    m, _ = W.config(2, with_state=False)
    Q = Sector_digit_sum(m, 0.0)
    S = sector(m, Q)
    assert S.dim == 7873260 and S.generated()
    rng = np.random.default_rng(7)
    x = W.random_state(S.dim, rng)
    y = S.matvec(t(m.theta), t(x))
    torch.cuda.synchronize()
    lab = osec.labels(m, Q)
    rows = np.unique(np.concatenate([np.arange(200), np.arange(S.dim - 200, S.dim),
                                     rng.choice(S.dim, 3000, replace=False)])).astype(np.int64)
    assert np.array_equal(S.labels().cpu().numpy()[rows], lab[rows])
    got = y[t(rows)].cpu().numpy()
    assert rel_err(got, osec.matvec(m, Q, x, lab=lab, rows=rows)) <= TOL_Z


def test_ring20_sz0_sector_whole_vector():
    """20-site ferrimagnetic ring, S_z = 0 sector (7,873,260 states), with the generated kernel the
    benchmark times: every packed row against the oracle (c128 at 1e-12; c64 at 2e-5 with the oracle fed
    the c64-rounded input), and every label (the packed digits) against the oracle's enumeration."""
    m, _ = W.config(2, with_state=False)
    Q = Sector_digit_sum(m, 0.0)
    S = sector(m, Q)
    assert S.generated() and S.generated(torch.complex64)
    lab = osec.labels(m, Q)
    assert np.array_equal(S.labels().cpu().numpy(), lab)
    x = W.random_state(S.dim, np.random.default_rng(8))
    y = S.matvec(t(m.theta), t(x)).cpu().numpy()
    e = rel_err(y, osec.matvec(m, Q, x, lab=lab))
    x32 = x.astype(np.complex64)
    y32 = S.matvec(t(m.theta.astype(np.float32)), t(x32)).cpu().numpy()
    e32 = rel_err(y32, osec.matvec(m, Q, x32.astype(np.complex128),
                                   theta=m.theta.astype(np.float32).astype(np.float64), lab=lab))
    print(f"sector whole vector: c128 {e:.2e}, c64 {e32:.2e}", flush=True)
    assert e <= TOL_Z and e32 <= TOL_C


def test_sector_edge_cases():
    """The two one-state sectors (all digits 0, all digits maximal), a sector of a one-site lattice, and
    argument errors."""
    from paper_2606_02169_amd.plan import Plan, Sector
    m, _ = W.config(2, reduced=8)
    qmax = sum(s.d - 1 for s in m.sites)
    plan = Plan.from_model(m)
    for Q in (0, qmax):
        S = Sector(plan, Q)
        assert S.dim == 1
        lab = osec.labels(m, Q)
        assert S.labels().cpu().tolist() == lab.tolist()
        x = np.array([0.3 - 0.4j])
        y = S.matvec(t(m.theta), t(x)).cpu().numpy()
        assert rel_err(y, osec.matvec(m, Q, x, lab=lab)) <= TOL_Z
    one = W.Model([W.spin_site(3)], [W.Term(0, W.OP_Z, -1, W.OP_Z, 0, 1.0)], np.array([0.7]))
    S1 = Sector(Plan.from_model(one), 2)
    assert S1.dim == 1 and S1.labels().cpu().tolist() == [2]
    from paper_2606_02169_amd import _lib as L
    with pytest.raises(L.MrmfError):
        Sector(plan, qmax + 1)
    S = Sector(plan, qmax // 2)
    with pytest.raises(ValueError):
        S.matvec(t(m.theta), t(np.zeros(S.dim + 1, dtype=np.complex128)))


def test_ring20_spin_flip_and_full_lanczos():
    """Headline ring (D = 60,466,176), sector Lanczos in the digit sums 12..18 (S_z = Q - 15).  The spin
    flip maps sector Q onto 30 - Q and reverses the field; the rest of H is flip-invariant and S_z is
    constant in a sector, so E_Q - E_{30-Q} = 2 h_z (Q - 15) exactly (h_z = 0.1).  The lowest of these
    sectors is Q = 14, below its neighbours; 100 full-basis Lanczos steps from the seeded vector (all
    sectors mixed) give a Ritz value above it (variational) by less than their residual."""
    from paper_2606_02169_amd.plan import Plan, Sector
    m, x = W.config(2)
    plan = Plan.from_model(m)
    th = t(m.theta)
    E = {}
    for Q in range(12, 19):
        S = Sector(plan, Q)
        assert S.generated()
        r = S.lanczos(th, t(W.random_state(S.dim, np.random.default_rng(100 + Q))), 100)["result"].cpu().numpy()
        assert r[2] <= 1e-8, (Q, r)
        E[Q] = r[0]
        print(Q, S.dim, repr(E[Q]), r[2], flush=True)
    for Q in (12, 13, 14):
        assert abs((E[Q] - E[30 - Q]) - 0.2 * (Q - 15)) <= 1e-9, Q
    assert E[14] < min(E[13], E[15])
    r = plan.lanczos(th, t(x), 100)["result"].cpu().numpy()
    print("full basis", repr(r[0]), r[2], flush=True)
    assert r[0] >= E[14] - 1e-9 and r[0] - E[14] <= r[2]


def test_ring20_sector_lanczos_certified_by_oracle():
    """Sector Lanczos at full size, certified by the oracle: the 20-site ring's digit-sum-14 sector (S_z =
    -1, 7,473,840 states, the sector of the ring's ground level), 100 steps with partial
    reorthogonalisation.  The Ritz vector is brought to the host and ||H_s u - theta u|| recomputed with
    the oracle's sector matvec (P H P^T through the full-basis row loop): it must equal the GPU's residual,
    and it pins the FP64 energy to an eigenvalue of H_s; the FP32-matvec form's energy is compared with
    that certified value (1e-5 relative)."""
    from paper_2606_02169_amd.plan import Plan, Sector
    m, _ = W.config(2, with_state=False)
    Q = 14
    lab = osec.labels(m, Q)
    S = Sector(Plan.from_model(m), Q)
    assert S.dim == lab.size
    th = t(m.theta)
    v0 = t(W.random_state(S.dim, np.random.default_rng(100 + Q)))
    out = {}
    for prec in ("z", "c_in_z"):
        r = S.lanczos(th, v0, 100, precision=prec, reorth="partial", theta_c=th.float())
        res = r["result"].cpu().numpy()
        u = r["u"].cpu().numpy()
        del r
        theta, r_gpu = float(res[0]), float(res[2])
        r_oracle = float(np.linalg.norm(osec.matvec(m, Q, u, lab=lab, rows=np.arange(lab.size)) - theta * u))
        nu = float(np.linalg.norm(u))
        print(f"{prec}: theta {theta!r} residual gpu {r_gpu:.3e} oracle {r_oracle:.3e} ||u|| {nu!r}", flush=True)
        assert int(res[3]) == 100 and abs(nu - 1.0) <= 1e-10
        assert abs(r_gpu - r_oracle) <= 1e-10 * r_oracle + 1e-13 * abs(theta)
        out[prec] = (theta, r_oracle)
    t64, r64 = out["z"]
    assert r64 <= 1e-8
    rel = abs(out["c_in_z"][0] - t64) / abs(t64)
    print(f"FP64 sector energy {t64!r} within {r64:.1e} of an eigenvalue; FP32 form rel {rel:.2e}", flush=True)
    assert rel <= 1e-5
