"""The plan-specialized matvec kernel (generated per plan, compiled with hiprtc) against the oracle:
the same tolerances as the generic kernel (c128 1e-12, c64 2e-5 relative), on random mixed spin/boson
models, several tilings, and the full-size workloads (sampled rows)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import mf
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
TOL_Z, TOL_C = 1e-12, 2e-5


def plan(model, kind="specialized", inner=0, **kw):
    from paper_2606_02169_amd.plan import Plan
    p = Plan.from_model(model, **kw)
    p.set_kernel(kind, inner)
    return p


def run(p, theta, x):
    dev = torch.device("cuda")
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    rd = torch.float64 if x.dtype == np.complex128 else torch.float32
    y = p.matvec(torch.as_tensor(theta, dtype=rd, device=dev), xt)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("seed", range(12))
def test_random_models_specialized(seed):
    rng = np.random.default_rng(3000 + seed)
    herm = seed % 4 != 0
    m = W.random_model(rng, n_sites=int(rng.integers(2, 8)), max_dim=40000, hermitian=herm,
                       n_params=int(rng.integers(1, 5)), n_terms=16)
    inner = int(rng.integers(0, 3))
    print(f"seed={seed} D={m.dim} sites={[s.d for s in m.sites]} terms={len(m.terms)} inner={inner}", flush=True)
    try:
        p = plan(m, inner=inner, require_hermitian=herm)
        p.prepare(torch.complex128)
    except Exception as e:           # the requested tile does not fit: let the library choose
        p = plan(m, inner=0, require_hermitian=herm)
    x = W.random_state(m.dim, rng)
    y = run(p, m.theta, x)
    info = p.kernel_info(torch.complex128)
    print(info, flush=True)
    assert info["kind"] == "specialized"
    assert rel_err(y, mf.matvec(m, x)) <= TOL_Z
    x32 = x.astype(np.complex64)
    assert rel_err(run(p, m.theta, x32), mf.matvec(m, x32.astype(np.complex128))) <= TOL_C


@pytest.mark.parametrize("k", [1, 5])
def test_small_configs_specialized(k):
    m, x = W.config(k)
    p = plan(m)
    assert rel_err(run(p, m.theta, x), mf.matvec(m, x)) <= TOL_Z
    assert p.kernel_info()["kind"] == "specialized"


def test_config2_full_size_specialized():
    m, x = W.config(2)
    p = plan(m)
    y = run(p, m.theta, x)
    print(p.kernel_info(), flush=True)
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([np.arange(300), np.arange(m.dim - 300, m.dim),
                                     rng.choice(m.dim, 4000, replace=False)])).astype(np.int64)
    assert rel_err(y[rows], mf.matvec(m, x, rows=rows)) <= TOL_Z
    assert np.all(np.isfinite(y))


def test_config3_full_size_specialized_c64():
    m, x = W.config(3)
    p = plan(m)
    y = run(p, m.theta, x)
    print(p.kernel_info(torch.complex64), flush=True)
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([np.arange(300), np.arange(m.dim - 300, m.dim),
                                     rng.choice(m.dim, 4000, replace=False)])).astype(np.int64)
    assert rel_err(y[rows], mf.matvec(m, x.astype(np.complex128), rows=rows)) <= TOL_C


def test_specialized_equals_generic_bitwise_structure():
    """Both kernels on the ferrimagnetic ring N=12: same result to rounding."""
    m, x = W.config(2, reduced=12)
    a = run(plan(m, "generic"), m.theta, x)
    b = run(plan(m, "specialized"), m.theta, x)
    assert rel_err(b, a) <= 1e-13


@pytest.mark.parametrize("k,inner,unrolled,U,cap", [(2, 6, 1, 4, 0), (2, 6, 1, 8, 0), (2, 7, 0, 4, 0),
                                                    (3, 5, 1, 4, 0), (3, 5, 2, 8, 0), (3, 6, 0, 8, 2)])
def test_list_form_full_size(k, inner, unrolled, U, cap):
    """List form at full size with several blocks per compute unit: sampled rows against the oracle,
    the whole vector against the masked form, and two runs bit-identical.  (A 128-bit store whose data
    registers were rewritten right after it once corrupted the real part of whole rows here.)"""
    from paper_2606_02169_amd.plan import Plan
    m, x = W.config(k)
    dev = torch.device("cuda")
    f32 = x.dtype == np.complex64
    rd = torch.float32 if f32 else torch.float64
    xt = torch.from_numpy(x).to(dev)
    th = torch.as_tensor(m.theta, dtype=rd, device=dev)
    ref = Plan.from_model(m)
    ref.set_kernel("specialized", 0, 0)
    y0 = ref.matvec(th, xt)
    p = Plan.from_model(m)
    p.set_kernel("specialized", inner, unrolled)
    p.set_tuning(variant=1, load_group=U, blocks_per_cu=cap)
    ya = p.matvec(th, xt).clone()
    yb = p.matvec(th, xt)
    torch.cuda.synchronize()
    print(p.kernel_info(xt.dtype), flush=True)
    assert torch.equal(ya, yb)
    tol = TOL_C if f32 else TOL_Z
    assert ((ya - y0).norm() / y0.norm()).item() <= (1e-6 if f32 else 1e-13)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([np.arange(300), np.arange(m.dim - 300, m.dim),
                                     rng.choice(m.dim, 4000, replace=False)])).astype(np.int64)
    yr = ya[torch.from_numpy(rows).to(dev)].cpu().numpy()
    assert rel_err(yr, mf.matvec(m, x.astype(np.complex128), rows=rows)) <= tol


def test_plan_autotune_and_cache(tmp_path, monkeypatch):
    """mrmf_plan_autotune on a reduced ring: the chosen shape reproduces the result, the cache entry is
    written and a second plan of the same structure takes it without a search."""
    from paper_2606_02169_amd.plan import Plan
    monkeypatch.setenv("MRMF_TUNE_CACHE", str(tmp_path / "tune.json"))
    m, x = W.config(2, reduced=14)
    dev = torch.device("cuda")
    xt = torch.from_numpy(x).to(dev)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device=dev)
    p = Plan.from_model(m)
    ent = p.autotune(th, xt)
    print(ent, flush=True)
    assert (tmp_path / "tune.json").exists()
    y = p.matvec(th, xt)
    torch.cuda.synchronize()
    assert rel_err(y.cpu().numpy(), mf.matvec(m, x)) <= TOL_Z
    q = Plan.from_model(m)
    ent2 = q.autotune(th, xt)
    assert ent2["key"] == ent["key"] and ent2["inner_sites"] == ent["inner_sites"]
    assert q.kernel_info()["inner_sites"] == ent["inner_sites"]


@pytest.mark.parametrize("seed,variant", [(0, 0), (1, 1), (2, 0), (3, 1), (4, 1), (5, 0)])
def test_wide_addressing_random_models(seed, variant):
    """64-bit addressing (a buffer resource per access at the super-tile's 64-bit base), forced on small
    random models: both forms, both element types, against the oracle."""
    rng = np.random.default_rng(5100 + seed)
    herm = seed % 3 != 0
    m = W.random_model(rng, n_sites=int(rng.integers(3, 8)), max_dim=40000, hermitian=herm,
                       n_params=int(rng.integers(1, 4)), n_terms=14)
    print(f"seed={seed} variant={variant} D={m.dim} sites={[s.d for s in m.sites]}", flush=True)
    p = plan(m, inner=0, require_hermitian=herm)
    p.set_tuning(variant=variant, addressing=1)
    x = W.random_state(m.dim, rng)
    assert rel_err(run(p, m.theta, x), mf.matvec(m, x)) <= TOL_Z
    assert p.kernel_info()["kind"] == "specialized"
    assert "RS(" in p.kernel_source()
    x32 = x.astype(np.complex64)
    assert rel_err(run(p, m.theta, x32), mf.matvec(m, x32.astype(np.complex128))) <= TOL_C


@pytest.mark.parametrize("variant", [0, 1])
def test_wide_addressing_beyond_2gib(variant):
    """The mixed (1/2)^6 (1)^6 (3/2)^6 ring (D = 24^6, 3.06 GB per complex128 vector, so 32-bit buffer
    offsets cannot reach it): the specialized kernel against the generic one on the whole vector and
    against the oracle on sampled rows, including both ends."""
    from paper_2606_02169_amd.plan import Plan
    m = W.paper_c2()
    dev = torch.device("cuda")
    rng = np.random.default_rng(77)
    x = W.random_state(m.dim, rng)
    xt = torch.from_numpy(x).to(dev)
    del x
    th = torch.as_tensor(m.theta, dtype=torch.float64, device=dev)
    g = Plan.from_model(m)
    g.set_kernel("generic")
    y0 = g.matvec(th, xt)
    p = Plan.from_model(m)
    p.set_kernel("specialized", 5, 0)
    p.set_tuning(variant=variant)
    y = p.matvec(th, xt)
    torch.cuda.synchronize()
    print(p.kernel_info(), flush=True)
    assert "RS(" in p.kernel_source()
    assert ((y - y0).norm() / y0.norm()).item() <= 1e-14
    del y0
    rows = np.unique(np.concatenate([np.arange(300), np.arange(m.dim - 300, m.dim),
                                     rng.choice(m.dim, 3000, replace=False)])).astype(np.int64)
    idx = torch.from_numpy(rows).to(dev)
    yr = y[idx].cpu().numpy()
    xr = xt.cpu().numpy()
    assert rel_err(yr, mf.matvec(m, xr, rows=rows)) <= TOL_Z


@pytest.mark.parametrize("k,inner,unrolled,variant,U", [(2, 7, 1, 1, 4), (2, 5, 2, 0, 0), (2, 6, 1, 0, 0),
                                                        (3, 5, 1, 1, 4), (3, 4, 1, 0, 0)])
def test_site0_unrolled_full_size(k, inner, unrolled, variant, U):
    """Site 0 unrolled with the low sites (MRMF_TUNE_UNROLL_TOP; the ring's closing bond (19, 0) and the
    torus's column wraps read LDS): full size against the default shape over the whole vector, sampled
    rows against the oracle, two runs bit-identical."""
    from paper_2606_02169_amd.plan import Plan
    m, x = W.config(k)
    dev = torch.device("cuda")
    f32 = x.dtype == np.complex64
    rd = torch.float32 if f32 else torch.float64
    xt = torch.from_numpy(x).to(dev)
    th = torch.as_tensor(m.theta, dtype=rd, device=dev)
    ref = Plan.from_model(m)
    ref.set_kernel("specialized", 0, 0)
    y0 = ref.matvec(th, xt)
    p = Plan.from_model(m)
    p.set_kernel("specialized", inner, unrolled)
    p.set_tuning(variant=variant, load_group=U, unroll_top=1)
    ya = p.matvec(th, xt).clone()
    yb = p.matvec(th, xt)
    torch.cuda.synchronize()
    info = p.kernel_info(xt.dtype)
    print(info, flush=True)
    assert info["kind"] == "specialized" and info["copies"] % m.sites[0].d == 0
    assert torch.equal(ya, yb)
    assert ((ya - y0).norm() / y0.norm()).item() <= (1e-6 if f32 else 1e-13)
    rng = np.random.default_rng(12)
    rows = np.unique(np.concatenate([np.arange(300), np.arange(m.dim - 300, m.dim),
                                     rng.choice(m.dim, 4000, replace=False)])).astype(np.int64)
    yr = ya[torch.from_numpy(rows).to(dev)].cpu().numpy()
    assert rel_err(yr, mf.matvec(m, x.astype(np.complex128), rows=rows)) <= (TOL_C if f32 else TOL_Z)


@pytest.mark.parametrize("variant", [0, 1])
def test_site0_unrolled_reduced_and_propagate(variant):
    """Reduced ring (N = 14) with site 0 unrolled: the whole vector against the oracle, and a propagation
    through the Chebyshev-step kernel of the same shape against the propagation oracle."""
    from oracle import propagate as oprop
    m, x = W.config(2, reduced=14)
    p = plan(m, inner=4)
    p.set_tuning(variant=variant, unroll_top=1)
    assert rel_err(run(p, m.theta, x), mf.matvec(m, x)) <= TOL_Z
    m8, x8 = W.config(2, reduced=8)
    q = plan(m8, inner=3)
    q.set_tuning(variant=variant, unroll_top=1)
    dev = torch.device("cuda")
    r = q.propagate(torch.from_numpy(m8.theta).to(dev), torch.from_numpy(x8).to(dev), 0.3, 2)
    q.prepare(torch.complex128)
    assert q.kernel_info()["kind"] == "specialized"
    assert rel_err(r["x"].cpu().numpy(), oprop.propagate(m8, x8, 0.3, 2)) <= 1e-11
