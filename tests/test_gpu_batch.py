"""Batched persistent form (mrmf_batch_matvec_c): every lattice block against the oracle (c64, 2e-5
relative per lattice and vector), hipGraph replays against the eager launch, and the autotuner."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import mf
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")
TOL_C = 2e-5


def build(models, xs, nvec=8):
    from paper_2606_02169_amd.plan import Batch, Plan
    plans = [Plan.from_model(m) for m in models]
    B = Batch(plans, nvec)
    X = torch.zeros(B.total_elems, dtype=torch.complex64, device=DEV)
    for b, x in enumerate(xs):
        B.block(X, b).copy_(torch.from_numpy(np.ascontiguousarray(x)).to(DEV))
    th = np.concatenate([m.theta for m in models]).astype(np.float32)
    return B, X, torch.from_numpy(th).to(DEV)


def check_all(B, models, xs, Y, rows=None):
    for b, (m, x) in enumerate(zip(models, xs)):
        yb = B.block(Y, b).cpu().numpy()
        for v in range(x.shape[1]):
            xv = x[:, v].astype(np.complex128)
            if rows is None:
                ref = mf.matvec(m, xv, theta=m.theta.astype(np.float32).astype(np.float64))
                got = yb[:, v]
            else:
                r = rows(m.dim)
                ref = mf.matvec(m, xv, theta=m.theta.astype(np.float32).astype(np.float64), rows=r)
                got = yb[r, v]
            assert rel_err(got, ref) <= TOL_C, (b, v)


def test_batch_reduced_against_oracle():
    models, xs = W.config(4, reduced=24)
    B, X, th = build(models, xs)
    Y = B.matvec(th, X)
    torch.cuda.synchronize()
    check_all(B, models, xs, Y)


@pytest.mark.parametrize("nvec", [1, 2, 4])
def test_batch_other_widths(nvec):
    rng = np.random.default_rng(100 + nvec)
    models = [W.random_model(rng, n_sites=int(rng.integers(2, 6)), max_dim=3000) for _ in range(7)]
    xs = [W.random_state(m.dim, rng, np.complex64, nvec=nvec) for m in models]
    B, X, th = build(models, xs, nvec)
    Y = B.matvec(th, X)
    torch.cuda.synchronize()
    check_all(B, models, xs, Y)


def test_batch_graph_replays_match_eager():
    models, xs = W.config(4, reduced=16)
    B, X, th = build(models, xs)
    Y_eager = B.matvec(th, X)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    Yg = torch.zeros_like(X)
    B.capture(th, X, Yg, s)
    for k in range(4):
        Yg.zero_()
        torch.cuda.synchronize()
        B.replay(s)
        s.synchronize()
        assert torch.equal(Yg, Y_eager), k
        X.mul_(1.0)                      # eager work between replays
        torch.cuda.synchronize()


def test_batch_autotune_keeps_results():
    models, xs = W.config(4, reduced=16)
    B, X, th = build(models, xs)
    Y0 = B.matvec(th, X).clone()
    Y = torch.empty_like(X)
    best = B.autotune(th, X, Y)
    print(best, flush=True)
    assert best["tile_rows_max"] > 0 and best["block"] % 64 == 0
    Y1 = B.matvec(th, X)
    torch.cuda.synchronize()
    assert rel_err(Y1.cpu().numpy(), Y0.cpu().numpy()) <= 1e-6


def test_batch_full_size_sampled():
    """256 open mixed-spin chains (N in 8..16, 2s in {1,2,3}, D <= 2^22), blocks of 8 vectors."""
    models, xs = W.config(4)
    dims = [m.dim for m in models]
    print(f"lattices {len(models)} sum D {sum(dims)} max D {max(dims)} min D {min(dims)}", flush=True)
    B, X, th = build(models, xs)
    B.set_shape(512, 512, "runs")
    Y = B.matvec(th, X).clone()
    B.set_shape(512, 512, "windows")
    assert torch.equal(B.matvec(th, X), Y)       # same rows, same arithmetic: identical bits
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)

    def rows(D):
        k = min(D, 300)
        return np.unique(np.concatenate([np.arange(min(D, 40)), np.arange(max(0, D - 40), D),
                                         rng.choice(D, k, replace=False)])).astype(np.int64)
    for b in range(0, len(models), 8):
        m, x = models[b], xs[b]
        yb = B.block(Y, b).cpu().numpy()
        r = rows(m.dim)
        for v in (0, 7):
            ref = mf.matvec(m, x[:, v].astype(np.complex128), theta=m.theta.astype(np.float32).astype(np.float64),
                            rows=r)
            assert rel_err(yb[r, v], ref) <= TOL_C, (b, v)


@pytest.mark.parametrize("schedule", ["runs", "windows", "xcd_chunk"])
@pytest.mark.parametrize("rmax,block", [(64, 64), (128, 128), (512, 256), (512, 512), (256, 512)])
def test_batch_every_shape(rmax, block, schedule):
    """Each launch shape (tiles of at most rmax rows held in LDS, block threads, work schedule) gives the
    oracle's result, including tiles smaller than the block (several tiles per item) and larger ones."""
    models, xs = W.config(4, reduced=12)
    B, X, th = build(models, xs)
    B.set_shape(rmax, block, schedule)
    assert B.shape()["schedule"] == schedule
    Y = B.matvec(th, X)
    torch.cuda.synchronize()
    check_all(B, models, xs, Y)


@pytest.mark.parametrize("nvec", [1, 2, 4])
def test_batch_vector_counts_and_alignment(nvec):
    """nvec = 1, 2, 4 against the oracle (rows moved in 8-byte words for one vector, 16-byte words
    otherwise); with two or more vectors a block that is only 8-byte aligned is refused, nothing launched."""
    from paper_2606_02169_amd import _lib as L
    from paper_2606_02169_amd.plan import _ptr, _stream
    rng = np.random.default_rng(40 + nvec)
    models = W.config(4, reduced=6, with_state=False)[0]
    xs = [W.random_state(m.dim, rng, np.complex64, nvec=nvec) for m in models]
    B, X, th = build(models, xs, nvec=nvec)
    B.set_shape(64 * 8 // nvec, 64, "windows")
    Y = B.matvec(th, X)
    torch.cuda.synchronize()
    check_all(B, models, xs, Y)
    Xs = torch.zeros(B.total_elems + 1, dtype=torch.complex64, device=DEV)[1:]   # 8-byte aligned only
    Ys = torch.empty(B.total_elems + 1, dtype=torch.complex64, device=DEV)[1:]
    st = L.lib().mrmf_batch_matvec_c(B._handle, _ptr(B.ws), _ptr(th), _ptr(Xs), _ptr(Ys), _stream(DEV))
    assert st == (L.MRMF_OK if nvec == 1 else L.MRMF_E_INVALID_ARG)
    torch.cuda.synchronize()


def test_parameter_sweep_in_one_launch():
    """A parameter sweep (Sec. VII: many couplings on one structure) as one batched launch: the same plan
    twelve times, each copy with its own couplings (J_z and h_z swept on the 10-site ferrimagnetic ring),
    the same 8 vectors in every block.  Every block against the oracle at its own couplings, and H x
    affine in theta along the sweep: y(J_z) - y(J_z0) proportional to J_z - J_z0 at fixed h_z (the
    diagonal channel's weight enters linearly)."""
    import dataclasses
    from paper_2606_02169_amd.plan import Batch, Plan
    base = W.ferrimagnetic_ring(10)                       # D = 7776; theta = [J_xy, J_z, D_si, h_z]
    jz = np.linspace(0.6, 1.8, 6)
    thetas = [np.array([1.0, j, 0.5, h]) for h in (0.0, 0.3) for j in jz]
    models = [dataclasses.replace(base, theta=t) for t in thetas]
    x = W.random_state(base.dim, np.random.default_rng(71), np.complex64, nvec=8)
    plan = Plan.from_model(base)
    B = Batch([plan] * len(models), 8)
    X = torch.zeros(B.total_elems, dtype=torch.complex64, device=DEV)
    for b in range(len(models)):
        B.block(X, b).copy_(torch.from_numpy(x).to(DEV))
    th = torch.from_numpy(np.concatenate(thetas).astype(np.float32)).to(DEV)
    Y = B.matvec(th, X)
    torch.cuda.synchronize()
    check_all(B, models, [x] * len(models), Y)
    ys = [B.block(Y, b).cpu().numpy().astype(np.complex128) for b in range(len(models))]
    for h in range(2):
        y0, y1 = ys[6 * h], ys[6 * h + 1]
        unit = (y1 - y0) / (jz[1] - jz[0])
        for k in range(2, 6):
            pred = y0 + (jz[k] - jz[0]) * unit
            assert rel_err(ys[6 * h + k], pred) <= 1e-5, (h, k)


def test_parameter_sweep_shared_input():
    """The same sweep with one shared input block (mrmf_batch_share_input: every lattice reads the block at
    the start of X, items tile by tile across the lattices): every output block equal, bit for bit, to the
    batch with a copy of the vectors per lattice, for each work schedule and two launch shapes, and against
    the oracle at its own couplings; a captured graph replays the shared mode."""
    import dataclasses
    from paper_2606_02169_amd.plan import Batch, Plan
    base = W.ferrimagnetic_ring(10)                       # D = 7776
    thetas = [np.array([1.0, j, 0.5, h]) for h in (0.0, 0.2, 0.4) for j in np.linspace(0.5, 1.5, 7)]
    models = [dataclasses.replace(base, theta=t) for t in thetas]
    x = W.random_state(base.dim, np.random.default_rng(72), np.complex64, nvec=8)
    plan = Plan.from_model(base)
    th = torch.from_numpy(np.concatenate(thetas).astype(np.float32)).to(DEV)
    ref_b = Batch([plan] * len(models), 8)
    Xc = torch.zeros(ref_b.total_elems, dtype=torch.complex64, device=DEV)
    xd = torch.from_numpy(x).to(DEV)
    for b in range(len(models)):
        ref_b.block(Xc, b).copy_(xd)
    Yref = ref_b.matvec(th, Xc)
    B = Batch([plan] * len(models), 8)
    B.share_input(True)
    assert B.input_elems < B.total_elems
    Xs = torch.zeros(B.input_elems, dtype=torch.complex64, device=DEV)
    Xs[: base.dim * 8].view(base.dim, 8).copy_(xd)
    for shape in ((512, 512), (256, 256)):
        for sched in ("runs", "windows", "xcd_chunk"):
            B.set_shape(*shape, sched)
            Y = torch.full((B.total_elems,), float("nan"), dtype=torch.complex64, device=DEV)
            B.matvec(th, Xs, Y)
            torch.cuda.synchronize()
            for b in range(len(models)):
                assert torch.equal(B.block(Y, b), ref_b.block(Yref, b)), (shape, sched, b)
    check_all(B, models, [x] * len(models), Y)
    s = torch.cuda.Stream(device=DEV)
    Yg = torch.full((B.total_elems,), float("nan"), dtype=torch.complex64, device=DEV)
    B.capture(th, Xs, Yg, s)
    for _ in range(2):
        Yg.fill_(float("nan"))
        torch.cuda.synchronize()
        B.replay(s)
        s.synchronize()
        for b in range(len(models)):
            assert torch.equal(B.block(Yg, b), ref_b.block(Yref, b)), b


def test_disorder_average_shared_input():
    """Shared input across lattices with the same local dimensions but different terms (a disorder average:
    10-site mixed chains, random J per bond, some with a next-nearest bond): each output block equal bit for
    bit to the batch with a copy per lattice, and against the oracle."""
    from workloads.model import Model, spin_site, xxz_bond_terms
    from paper_2606_02169_amd.plan import Batch, Plan
    rng = np.random.default_rng(73)
    sites = [spin_site(k) for k in (1, 2, 3, 1, 2, 3, 1, 2, 1, 2)]
    models = []
    for r in range(6):
        bonds = [(i, i + 1) for i in range(9)] + ([(0, 2), (5, 7)] if r % 2 else [])
        terms, theta = [], []
        for k, (i, j) in enumerate(bonds):
            terms += xxz_bond_terms(i, j, 2 * k, 2 * k + 1)
            theta += [rng.uniform(0.5, 1.5), rng.uniform(-1.0, 1.0)]
        models.append(Model(sites, terms, np.array(theta)))
    x = W.random_state(models[0].dim, np.random.default_rng(74), np.complex64, nvec=8)
    plans = [Plan.from_model(m) for m in models]
    th = torch.from_numpy(np.concatenate([m.theta for m in models]).astype(np.float32)).to(DEV)
    ref_b = Batch(plans, 8)
    Xc = torch.zeros(ref_b.total_elems, dtype=torch.complex64, device=DEV)
    xd = torch.from_numpy(x).to(DEV)
    for b in range(len(models)):
        ref_b.block(Xc, b).copy_(xd)
    Yref = ref_b.matvec(th, Xc)
    B = Batch(plans, 8)
    B.share_input(True)
    Xs = torch.zeros(B.input_elems, dtype=torch.complex64, device=DEV)
    Xs[: models[0].dim * 8].view(models[0].dim, 8).copy_(xd)
    for sched in ("runs", "windows", "xcd_chunk"):
        B.set_shape(256, 256, sched)
        Y = B.matvec(th, Xs)
        torch.cuda.synchronize()
        for b in range(len(models)):
            assert torch.equal(B.block(Y, b), ref_b.block(Yref, b)), (sched, b)
    check_all(B, models, [x] * len(models), Y)


def test_sweep_by_linearity():
    """Sweep (group products h_p X from one batched launch, then Y_k = sum_p theta_kp h_p X in one combining
    pass) against the direct batched products at each coupling vector (FP32 sums in another order: within
    2e-6 relative) and against the oracle in FP64; the group products equal the plan's matvec at unit
    couplings."""
    import dataclasses
    from paper_2606_02169_amd.plan import Batch, Plan, Sweep
    base = W.ferrimagnetic_ring(10)
    thetas = [np.array([1.0, j, 0.5, h]) for h in (0.0, 0.3, -0.2) for j in np.linspace(0.4, 1.6, 9)]
    models = [dataclasses.replace(base, theta=t) for t in thetas]
    x = W.random_state(base.dim, np.random.default_rng(75), np.complex64, nvec=8)
    plan = Plan.from_model(base)
    sw = Sweep(plan, 8)
    X = torch.zeros(sw.input_elems, dtype=torch.complex64, device=DEV)
    X[: sw.n].view(base.dim, 8).copy_(torch.from_numpy(x).to(DEV))
    th = torch.from_numpy(np.stack(thetas).astype(np.float32)).to(DEV)
    Y = sw.run(th, X)
    B = Batch([plan] * len(models), 8)
    B.share_input(True)
    Yd = B.matvec(th.reshape(-1), X)
    torch.cuda.synchronize()
    worst = 0.0
    for k in range(len(models)):
        a, b = sw.block(Y, k).cpu().numpy(), B.block(Yd, k).cpu().numpy()
        worst = max(worst, rel_err(a, b))
    print("sweep by linearity vs direct", worst, flush=True)
    assert worst <= 2e-6
    class _View:                                    # check_all reads blocks through .block
        def block(self, T, k):
            return sw.block(T, k)
    check_all(_View(), models, [x] * len(models), Y)
