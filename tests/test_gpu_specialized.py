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
