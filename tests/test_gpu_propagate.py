"""Time propagation (mrmf_propagate_z, Chebyshev expansion over the matrix-free matvec) against the
propagation oracle on random mixed spin/boson models, fixed and driven; at large D against the free-
fermion closed form and through the properties every exact propagation has (norm, energy, reversal)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle import propagate as oprop
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def mk(model, **kw):
    from paper_2606_02169_amd.plan import Plan
    return Plan.from_model(model, **kw)


@pytest.mark.parametrize("seed", range(6))
def test_propagate_random_models(seed):
    rng = np.random.default_rng(8100 + seed)
    m = W.random_model(rng, n_sites=int(rng.integers(2, 6)), max_dim=1500, n_params=int(rng.integers(1, 4)))
    x0 = W.random_state(m.dim, rng)
    dt, steps = float(rng.uniform(0.05, 0.6)), int(rng.integers(1, 5))
    print(f"seed={seed} D={m.dim} dt={dt} steps={steps}", flush=True)
    p = mk(m)
    r = p.propagate(t(m.theta), t(x0), dt, steps)
    ref = oprop.propagate(m, x0, dt, steps)
    print(r["n_terms"], r["bounds"], flush=True)
    assert rel_err(r["x"].cpu().numpy(), ref) <= 1e-11


def test_propagate_driven_and_in_place():
    """theta_s = theta (1 + 0.4 cos(Omega t_s)) held for each step (piecewise-constant drive); the
    result overwrites x0 in place; tight spectral bounds from the dense spectrum."""
    from oracle import kron
    rng = np.random.default_rng(8200)
    m = W.random_model(rng, n_sites=4, max_dim=900, n_params=3)
    x0 = W.random_state(m.dim, rng)
    steps, dt, om = 7, 0.3, 1.7
    thetas = np.stack([m.theta * (1 + 0.4 * np.cos(om * dt * s)) for s in range(steps)])
    ev = np.concatenate([np.linalg.eigvalsh(kron.dense_H(m, th)) for th in thetas])
    p = mk(m)
    x = t(x0)
    r = p.propagate(t(thetas), x, dt, steps, bounds=(ev.min() - 1e-6, ev.max() + 1e-6), out=x)
    assert r["x"].data_ptr() == x.data_ptr()
    ref = oprop.propagate(m, x0, dt, steps, thetas=thetas)
    assert rel_err(x.cpu().numpy(), ref) <= 1e-11


def test_magnon_closed_form_large():
    """Open spin-1/2 XX chain, N = 22 (D = 4,194,304): one up spin hops with amplitude J/2, so the
    propagated state is sum_k phi_k(n) phi_k(m) exp(-i eps_k t) on the one-magnon rows and exactly zero
    elsewhere."""
    N, J, tt, start = 22, 1.0, 3.0, 7
    m = W.xx_chain_in_field(N, J, 0.0)
    x0 = np.zeros(m.dim, dtype=np.complex128)
    x0[2 ** (N - start)] = 1.0
    p = mk(m)
    r = p.propagate(t(m.theta), t(x0), tt / 4, 4)
    x = r["x"].cpu().numpy()
    k = np.arange(1, N + 1)
    phi = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(k, k) * np.pi / (N + 1))
    amp = (phi * np.exp(-1j * J * np.cos(k * np.pi / (N + 1)) * tt)[:, None]).T @ phi[:, start - 1]
    rows = 2 ** (N - k)
    assert np.max(np.abs(x[rows] - amp)) <= 1e-12
    rest = np.ones(m.dim, dtype=bool)
    rest[rows] = False
    assert np.all(x[rest] == 0)


def test_full_size_ring_invariants():
    """20-site ferrimagnetic ring (D = 60,466,176, c128): norm and energy conserved, and propagating back
    returns the start vector."""
    m, x0 = W.config(2)
    p = mk(m)
    th = t(m.theta)
    xs = t(x0)
    fwd = p.propagate(th, xs, 0.05, 3)
    print("terms per step", fwd["n_terms"], fwd["bounds"], flush=True)
    x = fwd["x"]
    assert abs(torch.linalg.vector_norm(x).item() - torch.linalg.vector_norm(xs).item()) <= 1e-11
    e0 = torch.vdot(xs, p.matvec(th, xs)).real.item()
    e1 = torch.vdot(x, p.matvec(th, x)).real.item()
    assert abs(e1 - e0) <= 1e-10 * max(1.0, abs(e0))
    back = p.propagate(th, x, -0.05, 3)["x"]
    assert ((back - xs).norm() / xs.norm()).item() <= 1e-11
    rows = np.unique(np.random.default_rng(3).choice(m.dim, 2000, replace=False))
    assert np.abs(x[t(rows)].cpu().numpy() - x0[rows]).max() > 1e-4      # it did move


@pytest.mark.parametrize("k", [2, 3])
def test_fused_step_matches_two_pass(k):
    """The specialized kernel's fused Chebyshev step against the generic kernel's matvec + update on the
    reduced ring / torus (sampled against the oracle as well)."""
    m, x0 = W.config(k, reduced=3 if k == 3 else 14)
    x0 = x0.astype(np.complex128)
    a, b = mk(m), mk(m)
    b.set_kernel("generic")
    th = t(m.theta)
    tuned = a.autotune(th, t(x0), kernel="cheb", use_cache=False)
    print("cheb shape", tuned, flush=True)
    ra = a.propagate(th, t(x0), 0.2, 2)
    rb = b.propagate(th, t(x0), 0.2, 2)
    a.prepare(torch.complex128)
    assert a.kernel_info()["kind"] == "specialized" and b.kernel_info()["kind"] == "generic"
    xa, xb = ra["x"].cpu().numpy(), rb["x"].cpu().numpy()
    assert rel_err(xa, xb) <= 1e-13
    if m.dim <= 200000:
        assert rel_err(xa, oprop.propagate(m, x0, 0.2, 2)) <= 1e-11


@pytest.mark.parametrize("steps", [2, 7, 401])
def test_merged_steps_match_stepwise(steps):
    """A fixed H's steps taken as longer steps (the default) against one series per step and against the
    oracle; the merged run takes fewer Chebyshev terms in all.  401 steps of dt = 0.9 exceed what one
    merged series may take (its terms are capped), so the run is split into series of fewer steps with a
    shorter one at the end; the oracle there is one expm of the whole time 401 dt (the exponential of a
    fixed H composes), the per-step product being too slow on the host."""
    rng = np.random.default_rng(8400 + steps)
    m = W.random_model(rng, n_sites=4, max_dim=400 if steps > 100 else 1200, n_params=2)
    x0 = W.random_state(m.dim, rng)
    dt = 0.9 if steps > 100 else 0.35
    p = mk(m)
    merged = p.propagate(t(m.theta), t(x0), dt, steps)
    p.set_tuning(cheb_merge=0)
    stepwise = p.propagate(t(m.theta), t(x0), dt, steps, bounds=merged["bounds"])
    ref = oprop.propagate(m, x0, dt * steps, 1) if steps > 100 else oprop.propagate(m, x0, dt, steps)
    xm, xs = merged["x"].cpu().numpy(), stepwise["x"].cpu().numpy()
    print(f"steps {steps}: terms merged {merged['n_terms']} stepwise {stepwise['n_terms']}, "
          f"bounds {merged['bounds']}, errors {rel_err(xm, ref):.2e} / {rel_err(xs, ref):.2e}", flush=True)
    assert rel_err(xm, ref) <= 1e-11 and rel_err(xs, ref) <= 1e-9
    assert merged["n_terms"] < stepwise["n_terms"]


def test_propagate_errors():
    from paper_2606_02169_amd import _lib as L
    m = W.xx_chain_in_field(4, 1.0, 0.2)
    p = mk(m)
    x = t(W.random_state(m.dim, np.random.default_rng(1)))
    with pytest.raises(Exception):
        p.propagate(t(m.theta), x, 0.1, 1, bounds=(1.0, 1.0))
    nh = W.Model([W.spin_site(1)], [W.Term(0, W.OP_RAISE, -1, W.OP_Z, 0, 1.0)], np.ones(1))
    q = mk(nh, require_hermitian=False)
    with pytest.raises(Exception):
        q.propagate(t(nh.theta), t(np.array([1, 0], dtype=np.complex128)), 0.1, 1, bounds=(-2.0, 2.0))
    nb = ctypes.c_size_t()
    L.call("mrmf_propagate_scratch_bytes", p._handle, ctypes.byref(nb))
    small = torch.empty(int(nb.value) - 256, dtype=torch.uint8, device=DEV)
    y = torch.empty_like(x)
    th = t(m.theta)
    st = L.lib().mrmf_propagate_z(p._handle, ctypes.c_void_p(p.ws.data_ptr()), ctypes.c_void_p(th.data_ptr()),
                                   0, 0.1, 1, -5.0, 5.0, 1e-12, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(small.data_ptr()), small.numel(),
                                   None, None)
    assert st == L.MRMF_E_WORKSPACE


def test_propagate_zero_steps_and_zero_time():
    m = W.xx_chain_in_field(6, 1.0, 0.3)
    x0 = W.random_state(m.dim, np.random.default_rng(2))
    p = mk(m)
    r = p.propagate(t(m.theta), t(x0), 0.3, 0)
    assert np.array_equal(r["x"].cpu().numpy(), x0)                 # zero steps: a copy
    r = p.propagate(t(m.theta), t(x0), 0.0, 3, bounds=(-5.0, 5.0))
    assert r["n_terms"] == 1
    assert np.array_equal(r["x"].cpu().numpy(), x0)                 # dt = 0: the identity, exactly


# ------------------------------------------------------------------ Gershgorin spectral bounds
def gershgorin_sparse(m, theta=None):
    """Gershgorin ends of the oracle's sparse H: min / max over rows of H_FF -+ sum_{F' != F} |H_FF'|."""
    from oracle import kron
    H = kron.sparse_H(m, theta).tocsr()
    d = H.diagonal()
    R = np.asarray(abs(H).sum(axis=1)).ravel() - np.abs(d)
    return float((d.real - R).min()), float((d.real + R).max())


def gershgorin_ring_dp(N, jxy=1.0, jz=1.2, dsi=0.5, hz=0.1):
    """Gershgorin ends of the alternating s=1/2 / s=1 XXZ ring by max-plus (min-plus) transfer matrices:
    each row's diagonal and hop radius are sums of site and bond functions of the spins m_i, so the
    extreme ends are closed walks around the ring, with S_+|m-1> = sqrt(s(s+1) - m(m-1)) |m>."""
    spins = [0.5 if i % 2 == 0 else 1.0 for i in range(N)]
    ms = [np.arange(-s, s + 1) for s in spins]

    def up(s, m):      # <m|S_+|m-1>, zero when m - 1 < -s
        return np.sqrt(s * (s + 1) - m * (m - 1)) if m - 1 >= -s else 0.0

    def dn(s, m):      # <m|S_-|m+1>, zero when m + 1 > s
        return np.sqrt(s * (s + 1) - m * (m + 1)) if m + 1 <= s else 0.0

    def site(i, m):
        return hz * m + (dsi * m * m if i % 2 == 1 else 0.0)

    ends = []
    for sign in (-1.0, 1.0):
        mats = []
        for i in range(N):
            j, si, sj = (i + 1) % N, spins[i], spins[(i + 1) % N]
            A = np.empty((len(ms[i]), len(ms[j])))
            for a, mi in enumerate(ms[i]):
                for b, mj in enumerate(ms[j]):
                    rad = 0.5 * abs(jxy) * (up(si, mi) * dn(sj, mj) + dn(si, mi) * up(sj, mj))
                    A[a, b] = site(i, mi) + jz * mi * mj + sign * rad
            mats.append(sign * A)          # maximise sign * (diag + sign * R)
        best = -np.inf
        for a0 in range(len(ms[0])):       # closed walks through each state of site 0
            v = np.full(len(ms[0]), -np.inf)
            v[a0] = 0.0
            for A in mats:
                v = np.max(v[:, None] + A, axis=0)
            best = max(best, v[a0])
        ends.append(sign * best)
    return ends[0], ends[1]


def test_spectral_bounds_match_gershgorin():
    """Reduced rings and the 20-site ring (D = 60,466,176) against the max-plus ends, a reduced ring and
    two spin-boson models against the sparse oracle matrix (no two channels share an entry in these
    models)."""
    from paper_2606_02169_amd.plan import Plan
    for N in (8, 20):
        m, _ = W.config(2, reduced=N if N < 20 else 0, with_state=False)
        lo, hi = mk(m).spectral_bounds(t(m.theta))
        rlo, rhi = gershgorin_ring_dp(N)
        print(N, (lo, hi), (rlo, rhi), flush=True)
        assert abs(lo - rlo) <= 1e-12 * abs(rlo) and abs(hi - rhi) <= 1e-12 * abs(rhi)
        if N == 8:
            slo, shi = gershgorin_sparse(m)
            assert abs(lo - slo) <= 1e-12 * abs(slo) and abs(hi - shi) <= 1e-12 * abs(shi)
    tc = W.tavis_cummings(4, 10, 1.0, 1.0, np.random.default_rng(5))
    lo, hi = Plan.from_model(tc).spectral_bounds(t(tc.theta))
    slo, shi = gershgorin_sparse(tc)
    assert abs(lo - slo) <= 1e-12 * max(1.0, abs(slo)) and abs(hi - shi) <= 1e-12 * max(1.0, abs(shi))
    # two 40-level modes and a spin: the term tables exceed what the kernel tabulates in LDS, so its rows
    # evaluate their factors
    from workloads.model import OP_LOWER, OP_RAISE, OP_Z, Model, Term, boson_site, spin_site
    tb = Model([boson_site(39), spin_site(1), boson_site(39)],
               [Term(0, OP_RAISE, 2, OP_LOWER, 0, 0.7 + 0.2j), Term(0, OP_LOWER, 2, OP_RAISE, 0, 0.7 - 0.2j),
                Term(0, OP_LOWER, 1, OP_RAISE, 1, 1.0), Term(0, OP_RAISE, 1, OP_LOWER, 1, 1.0),
                Term(1, OP_RAISE, -1, OP_Z, 1, 0.3), Term(1, OP_LOWER, -1, OP_Z, 1, 0.3),
                Term(0, OP_Z, -1, OP_Z, 2, 1.0), Term(2, OP_Z, -1, OP_Z, 2, 1.3), Term(0, OP_Z, 2, OP_Z, 3, 0.05)],
               np.array([1.0, 0.4, 0.9, 0.5]))
    lo, hi = Plan.from_model(tb).spectral_bounds(t(tb.theta))
    slo, shi = gershgorin_sparse(tb)
    print("two bosons", (lo, hi), (slo, shi), flush=True)
    assert abs(lo - slo) <= 1e-12 * max(1.0, abs(slo)) and abs(hi - shi) <= 1e-12 * max(1.0, abs(shi))


@pytest.mark.parametrize("seed", range(6))
def test_spectral_bounds_contain_spectrum(seed):
    """Random mixed models (channels may share entries, so the channel sum can exceed the row sum): the
    bounds contain the oracle's Gershgorin interval, hence the spectrum; propagation with them matches the
    oracle."""
    from oracle import kron
    rng = np.random.default_rng(8300 + seed)
    m = W.random_model(rng, n_sites=int(rng.integers(2, 6)), max_dim=1200, n_params=int(rng.integers(1, 4)))
    p = mk(m)
    lo, hi = p.spectral_bounds(t(m.theta))
    slo, shi = gershgorin_sparse(m)
    ev = np.linalg.eigvalsh(kron.dense_H(m))
    tol = 1e-12 * max(1.0, abs(slo), abs(shi))
    print(seed, m.dim, (lo, hi), (slo, shi), (ev[0], ev[-1]), flush=True)
    assert lo <= slo + tol and hi >= shi - tol
    assert lo <= ev[0] + tol and hi >= ev[-1] - tol
    x0 = W.random_state(m.dim, rng)
    r = p.propagate(t(m.theta), t(x0), 0.4, 2)
    assert r["bounds"][0] <= lo and r["bounds"][1] >= hi
    assert rel_err(r["x"].cpu().numpy(), oprop.propagate(m, x0, 0.4, 2)) <= 1e-11


def test_spectral_bounds_driven_and_fewer_terms():
    """A piecewise drive takes the extreme ends over its steps; on the reduced ring the Gershgorin default
    needs fewer Chebyshev terms than the norm bound for the same result."""
    rng = np.random.default_rng(8400)
    m = W.random_model(rng, n_sites=4, max_dim=900, n_params=3)
    steps = 5
    thetas = np.stack([m.theta * (1 + 0.5 * np.cos(1.3 * s)) for s in range(steps)])
    p = mk(m)
    each = [p.spectral_bounds(t(th)) for th in thetas]
    x0 = W.random_state(m.dim, rng)
    r = p.propagate(t(thetas), t(x0), 0.3, steps)
    assert r["bounds"][0] <= min(e[0] for e in each) and r["bounds"][1] >= max(e[1] for e in each)
    assert rel_err(r["x"].cpu().numpy(), oprop.propagate(m, x0, 0.3, steps, thetas=thetas)) <= 1e-11
    m, x0 = W.config(2, reduced=10)
    p = mk(m)
    g = p.propagate(t(m.theta), t(x0), 0.5, 2)
    n = p.propagate(t(m.theta), t(x0), 0.5, 2, bounds="norm")
    print("terms", g["n_terms"], n["n_terms"], g["bounds"], n["bounds"], flush=True)
    assert g["n_terms"] < n["n_terms"]
    ref = oprop.propagate(m, x0, 0.5, 2)
    assert rel_err(g["x"].cpu().numpy(), ref) <= 1e-11 and rel_err(n["x"].cpu().numpy(), ref) <= 1e-11


@pytest.mark.parametrize("driven", [False, True])
def test_sector_propagation_against_oracle(driven):
    """Propagation inside a fixed-S_z sector of the 6-site ferrimagnetic ring (M = 1/2, fixed couplings,
    and a piecewise-constant drive of J_z and h_z): against exp(-i dt H_s) applied step by step, H_s the
    oracle's dense Kronecker H restricted to the sector's states (the oracle's labels), i.e. P H P^T."""
    from scipy.linalg import expm
    from oracle import kron
    from oracle import sector as osec
    from paper_2606_02169_amd.plan import Plan, Sector
    m = W.ferrimagnetic_ring(6)
    Q = Sector.digit_sum_of(m.sites, 0.5)
    lab = osec.labels(m, Q)
    steps, dt = 5, 0.35
    scale = [np.array([1.0, 1 + 0.3 * np.sin(1.3 * s), 1.0, 1 + 0.5 * np.cos(0.7 * s)]) if driven else np.ones(4)
             for s in range(steps)]
    thetas = np.stack([m.theta * f for f in scale])
    x0 = W.random_state(lab.size, np.random.default_rng(8400 + driven))
    S = Sector(Plan.from_model(m), Q)
    r = S.propagate(t(thetas) if driven else t(m.theta), t(x0), dt, steps)
    ref = x0.astype(np.complex128)
    for th in thetas:
        ref = expm(-1j * dt * kron.dense_H(m, th)[np.ix_(lab, lab)]) @ ref
    print(f"sector dim {lab.size}, terms {r['n_terms']}, rel err {rel_err(r['x'].cpu().numpy(), ref):.2e}", flush=True)
    assert rel_err(r["x"].cpu().numpy(), ref) <= 1e-11


def test_sector_propagation_equals_full_basis():
    """H keeps the digit sum, so a vector supported on a sector stays there: propagating it in the full
    basis (the 12-site ferrimagnetic ring, D = 46,656, the plan's fused kernel) gives zero outside the
    sector and, on its rows, the sector propagation of the packed vector (the sector kernel and the
    two-pass update; rows located by the oracle's labels), with the same spectral bounds."""
    from oracle import sector as osec
    from paper_2606_02169_amd.plan import Plan, Sector
    m, _ = W.config(2, reduced=12)
    Q = Sector.digit_sum_of(m.sites, 0.0)
    lab = osec.labels(m, Q)
    xs = W.random_state(lab.size, np.random.default_rng(8500))
    xf = np.zeros(m.dim, dtype=np.complex128)
    xf[lab] = xs
    p = Plan.from_model(m)
    S = Sector(p, Q)
    th = t(m.theta)
    rs = S.propagate(th, t(xs), 0.2, 6)
    rf = p.propagate(th, t(xf), 0.2, 6, bounds=rs["bounds"])
    ys, yf = rs["x"].cpu().numpy(), rf["x"].cpu().numpy()
    print(f"sector dim {lab.size} of {m.dim}; terms {rs['n_terms']} / {rf['n_terms']}; outside max "
          f"{np.max(np.abs(np.delete(yf, lab))):.2e}; rel diff {rel_err(yf[lab], ys):.2e}", flush=True)
    assert rs["n_terms"] == rf["n_terms"]
    assert np.max(np.abs(np.delete(yf, lab))) <= 1e-13
    assert rel_err(yf[lab], ys) <= 1e-12
    assert abs(np.linalg.norm(ys) - 1.0) <= 1e-12


def test_sector_propagation_fused_matches_two_pass():
    """The sector's generated kernel with the Chebyshev-step epilogue (one launch per term) against the
    sector matvec plus a separate update (the plan's cheb_fused = 0 when the sector is made): the same
    state to rounding, on the 12-site ring's S_z = 0 sector, fixed couplings and a drive."""
    from paper_2606_02169_amd.plan import Plan, Sector
    m, _ = W.config(2, reduced=12)
    Q = Sector.digit_sum_of(m.sites, 0.0)
    pf, p2 = Plan.from_model(m), Plan.from_model(m)
    p2.set_tuning(cheb_fused=0)
    Sf, S2 = Sector(pf, Q), Sector(p2, Q)
    assert Sf.generated()
    xs = t(W.random_state(Sf.dim, np.random.default_rng(8600)))
    drive = np.stack([m.theta * (1 + 0.2 * np.sin(0.9 * s)) for s in range(3)])
    for th, steps in ((t(m.theta), 5), (t(drive), 3)):
        rf = Sf.propagate(th, xs, 0.15, steps)
        r2 = S2.propagate(th, xs, 0.15, steps, bounds=rf["bounds"])
        e = rel_err(rf["x"].cpu().numpy(), r2["x"].cpu().numpy())
        print(f"steps {steps}: terms {rf['n_terms']} / {r2['n_terms']}, fused vs two-pass {e:.2e}", flush=True)
        assert rf["n_terms"] == r2["n_terms"] and e <= 1e-13


def sector_gershgorin_dense(m, lab, theta=None):
    """Gershgorin ends of P H P^T from the oracle's dense Kronecker H restricted to the sector's states."""
    from oracle import kron
    Hs = kron.dense_H(m, theta)[np.ix_(lab, lab)]
    d = np.diag(Hs)
    R = np.abs(Hs).sum(axis=1) - np.abs(d)
    return float((d.real - R).min()), float((d.real + R).max()), np.linalg.eigvalsh(Hs)


@pytest.mark.parametrize("case", ["ring6_half", "ring8_zero", "ring8_generic", "spin1_ring6", "mixed_ring6",
                                  "tavis_cummings", "two_bosons"])
def test_sector_spectral_bounds_match_gershgorin(case):
    """mrmf_sector_spectral_bounds against the Gershgorin ends of the oracle's dense H restricted to the
    sector (no two channels share an entry in these models; digits from the packed-digit words, or by
    unranking for a sector made in generic mode), hence containing the sector's spectrum, and inside the
    plan's bounds (every sector row is a row of H, with a subset of its off-diagonal entries)."""
    from oracle import sector as osec
    from paper_2606_02169_amd.plan import Plan, Sector
    if case == "tavis_cummings":
        m = W.tavis_cummings(4, 6, 1.0, 0.7, np.random.default_rng(5))
        Q = 5
    elif case == "two_bosons":        # two 40-level modes and a spin between them: term tables too large to
        from workloads.model import OP_LOWER, OP_RAISE, OP_Z, Model, Term, boson_site, spin_site
        m = Model([boson_site(39), spin_site(1), boson_site(39)],   # tabulate, so rows evaluate factors
                  [Term(0, OP_RAISE, 2, OP_LOWER, 0, 0.7 + 0.2j), Term(0, OP_LOWER, 2, OP_RAISE, 0, 0.7 - 0.2j),
                   Term(0, OP_LOWER, 1, OP_RAISE, 1, 1.0), Term(0, OP_RAISE, 1, OP_LOWER, 1, 1.0),
                   Term(0, OP_Z, -1, OP_Z, 2, 1.0), Term(2, OP_Z, -1, OP_Z, 2, 1.3), Term(1, OP_Z, -1, OP_Z, 3, 1.0),
                   Term(0, OP_Z, 2, OP_Z, 3, 0.05)],
                  np.array([1.0, 0.4, 0.9, 0.5]))
        Q = 30
    else:
        m = {"ring6_half": lambda: W.ferrimagnetic_ring(6), "ring8_zero": lambda: W.ferrimagnetic_ring(8),
             "ring8_generic": lambda: W.ferrimagnetic_ring(8),
             "spin1_ring6": lambda: W.staggered_xxz_ring([2] * 6),
             "mixed_ring6": lambda: W.staggered_xxz_ring([1, 1, 2, 2, 3, 3])}[case]()
        Q = Sector.digit_sum_of(m.sites, 0.5 if case == "ring6_half" else 0.0)
    lab = osec.labels(m, Q)
    p = Plan.from_model(m)
    if case == "ring8_generic":       # a sector made from a plan in generic mode holds no packed digits: the
        p.set_kernel("generic")       # bounds kernel unranks its rows
    S = Sector(p, Q)
    assert S.dim == lab.size
    lo, hi = S.spectral_bounds(t(m.theta))
    slo, shi, ev = sector_gershgorin_dense(m, lab)
    plo, phi = p.spectral_bounds(t(m.theta))
    tol = 1e-12 * max(1.0, abs(slo), abs(shi))
    print(case, lab.size, (lo, hi), (slo, shi), (ev[0], ev[-1]), (plo, phi), flush=True)
    assert abs(lo - slo) <= tol and abs(hi - shi) <= tol
    assert lo <= ev[0] + tol and hi >= ev[-1] - tol
    assert plo <= lo + tol and phi >= hi - tol


def test_sector_spectral_bounds_default_and_fewer_terms():
    """Sector propagation defaults to the sector's own bounds (extreme ends over a drive's steps): on the
    12-site ring's S_z = 0 sector they are no wider than the plan's and need no more Chebyshev terms, for
    the same state; on the 6-site ring's M = 1/2 sector the driven result matches exp(-i dt H_s) step by
    step."""
    from scipy.linalg import expm
    from oracle import kron
    from oracle import sector as osec
    from paper_2606_02169_amd.plan import Plan, Sector
    m, _ = W.config(2, reduced=12)
    p = Plan.from_model(m)
    S = Sector(p, Sector.digit_sum_of(m.sites, 0.0))
    th = t(m.theta)
    xs = t(W.random_state(S.dim, np.random.default_rng(8700)))
    rs = S.propagate(th, xs, 0.5, 2)
    rp = S.propagate(th, xs, 0.5, 2, bounds=p.spectral_bounds(th))
    lo, hi = S.spectral_bounds(th)
    print("sector bounds", rs["bounds"], "plan bounds", rp["bounds"], "terms", rs["n_terms"], rp["n_terms"],
          flush=True)
    assert rs["bounds"][0] <= lo and rs["bounds"][1] >= hi
    assert rs["bounds"][1] - rs["bounds"][0] <= rp["bounds"][1] - rp["bounds"][0]
    assert rs["n_terms"] <= rp["n_terms"]
    assert rel_err(rs["x"].cpu().numpy(), rp["x"].cpu().numpy()) <= 1e-11
    m = W.ferrimagnetic_ring(6)
    Q = Sector.digit_sum_of(m.sites, 0.5)
    lab = osec.labels(m, Q)
    S = Sector(Plan.from_model(m), Q)
    steps, dt = 4, 0.3
    thetas = np.stack([m.theta * np.array([1.0, 1 + 0.4 * np.sin(s), 1.0, 1 + 0.6 * np.cos(s)]) for s in range(steps)])
    each = [S.spectral_bounds(t(x)) for x in thetas]
    x0 = W.random_state(lab.size, np.random.default_rng(8701))
    r = S.propagate(t(thetas), t(x0), dt, steps)
    assert r["bounds"][0] <= min(e[0] for e in each) and r["bounds"][1] >= max(e[1] for e in each)
    ref = x0.astype(np.complex128)
    for x in thetas:
        ref = expm(-1j * dt * kron.dense_H(m, x)[np.ix_(lab, lab)]) @ ref
    assert rel_err(r["x"].cpu().numpy(), ref) <= 1e-11


# ------------------------------------------------------------------ bounds over many coupling vectors
def drive_rows(theta, S, rng):
    """S coupling vectors around theta, some of the couplings changing sign."""
    return np.stack([theta * rng.uniform(-1.5, 1.5, size=theta.size) for _ in range(S)])


@pytest.mark.parametrize("seed", range(4))
def test_spectral_bounds_many_random_models(seed):
    """One pass over the rows for S coupling vectors (mrmf_spectral_bounds_many) against the extremes of
    the per-vector device bounds and of the oracle matrix's Gershgorin ends per vector."""
    rng = np.random.default_rng(8800 + seed)
    m = W.random_model(rng, n_sites=int(rng.integers(2, 6)), max_dim=1200, n_params=int(rng.integers(1, 4)))
    p = mk(m)
    th = drive_rows(m.theta, 5, rng)
    lo, hi = p.spectral_bounds(t(th))
    each = [p.spectral_bounds(t(r)) for r in th]
    ref = [gershgorin_sparse(m, r) for r in th]
    elo, ehi = min(e[0] for e in each), max(e[1] for e in each)
    slo, shi = min(e[0] for e in ref), max(e[1] for e in ref)
    tol = 1e-12 * max(1.0, abs(elo), abs(ehi))
    print(seed, m.dim, m.n_params, (lo, hi), (elo, ehi), (slo, shi), flush=True)
    assert abs(lo - elo) <= tol and abs(hi - ehi) <= tol
    assert lo <= slo + tol and hi >= shi - tol


def test_spectral_bounds_many_full_ring_and_sector():
    """The 20-site ring (D = 60,466,176) and its S_z = 0 sector with a drive of 6 coupling vectors: one pass
    against six; stride 0 repeats one vector; a plan whose term tables are too large for the one-pass form
    is answered per vector."""
    from paper_2606_02169_amd import _lib as L
    from paper_2606_02169_amd.plan import Plan, Sector, _ptr, _stream
    m, _ = W.config(2, with_state=False)
    rng = np.random.default_rng(8900)
    th = drive_rows(m.theta, 6, rng)
    p = Plan.from_model(m)
    S = Sector(p, Sector.digit_sum_of(m.sites, 0.0))
    for obj in (p, S):
        lo, hi = obj.spectral_bounds(t(th))
        each = [obj.spectral_bounds(t(r)) for r in th]
        elo, ehi = min(e[0] for e in each), max(e[1] for e in each)
        print(type(obj).__name__, (lo, hi), (elo, ehi), flush=True)
        assert abs(lo - elo) <= 1e-12 * abs(elo) and abs(hi - ehi) <= 1e-12 * abs(ehi)
    # stride 0: the same vector three times
    nb = ctypes.c_size_t()
    L.call("mrmf_spectral_bounds_scratch_bytes", p._handle, ctypes.byref(nb))
    scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=DEV)
    out = torch.empty(2, dtype=torch.float64, device=DEV)
    t0 = t(th[0])
    L.call("mrmf_spectral_bounds_many", p._handle, _ptr(p.ws), _ptr(t0), 0, 3, _ptr(out), _ptr(scratch), nb.value,
           _stream(DEV))
    one = p.spectral_bounds(t0)
    got = out.cpu().tolist()
    assert abs(got[0] - one[0]) <= 1e-12 * abs(one[0]) and abs(got[1] - one[1]) <= 1e-12 * abs(one[1])
    # too large for the one-pass form: the binding falls back to one pass per vector
    from workloads.model import OP_LOWER, OP_RAISE, OP_Z, Model, Term, boson_site, spin_site
    tb = Model([boson_site(39), spin_site(1), boson_site(39)],
               [Term(0, OP_RAISE, 2, OP_LOWER, 0, 0.7), Term(0, OP_LOWER, 2, OP_RAISE, 0, 0.7),
                Term(0, OP_Z, -1, OP_Z, 1, 1.0), Term(1, OP_Z, -1, OP_Z, 1, 1.0)], np.array([1.0, 0.5]))
    pb = Plan.from_model(tb)
    thb = drive_rows(tb.theta, 3, rng)
    st = L.lib().mrmf_spectral_bounds_many(pb._handle, _ptr(pb.ws), _ptr(t(thb)), 2, 3, _ptr(out), _ptr(scratch),
                                           nb.value, _stream(DEV))
    assert st == L.MRMF_E_UNSUPPORTED
    lo, hi = pb.spectral_bounds(t(thb))
    ref = [gershgorin_sparse(tb, r) for r in thb]
    assert abs(lo - min(e[0] for e in ref)) <= 1e-12 * max(1.0, abs(lo))
    assert abs(hi - max(e[1] for e in ref)) <= 1e-12 * max(1.0, abs(hi))


def test_sector_spectral_bounds_many_against_dense():
    """The sector's one-pass ends over a drive against the Gershgorin ends of the oracle's dense P H P^T
    per coupling vector, and a driven sector propagation with those bounds against exp(-i dt H_s) step by
    step."""
    from scipy.linalg import expm
    from oracle import kron
    from oracle import sector as osec
    from paper_2606_02169_amd.plan import Plan, Sector
    m = W.staggered_xxz_ring([1, 1, 2, 2, 3, 3])
    Q = Sector.digit_sum_of(m.sites, 0.0)
    lab = osec.labels(m, Q)
    S = Sector(Plan.from_model(m), Q)
    th = drive_rows(m.theta, 5, np.random.default_rng(9000))
    lo, hi = S.spectral_bounds(t(th))
    ref = [sector_gershgorin_dense(m, lab, r)[:2] for r in th]
    slo, shi = min(e[0] for e in ref), max(e[1] for e in ref)
    print((lo, hi), (slo, shi), flush=True)
    assert abs(lo - slo) <= 1e-12 * max(1.0, abs(slo)) and abs(hi - shi) <= 1e-12 * max(1.0, abs(shi))
    x0 = W.random_state(lab.size, np.random.default_rng(9001))
    r = S.propagate(t(th), t(x0), 0.2, th.shape[0])
    assert r["bounds"][0] <= lo and r["bounds"][1] >= hi
    ref_x = x0.astype(np.complex128)
    for x in th:
        ref_x = expm(-1j * 0.2 * kron.dense_H(m, x)[np.ix_(lab, lab)]) @ ref_x
    assert rel_err(r["x"].cpu().numpy(), ref_x) <= 1e-11
