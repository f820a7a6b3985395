"""GPU parity of the matvec kernels against the oracle (through the C ABI).

Tolerances: c128 relative 2-norm error <= 1e-12, c64 <= 2e-5 (the c64 kernel is compared with the
FP64 oracle applied to the c64 input upcast exactly); source indices bit-exact."""
import numpy as np
import pytest
import torch

import workloads as W
from workloads.model import OP_LOWER, OP_RAISE, OP_Z, Model, Term, boson_site, spin_site
from oracle import mf
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu

TOL_Z = 1e-12
TOL_C = 2e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2606_02169_amd import build as _b  # noqa: F401  (import check only)


def Plan(model, **kw):
    from paper_2606_02169_amd.plan import Plan as P
    return P.from_model(model, **kw)


def gpu_matvec(plan, theta, x):
    dev = torch.device("cuda")
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    rd = torch.float64 if x.dtype == np.complex128 else torch.float32
    th = torch.as_tensor(theta, dtype=rd, device=dev)
    y = plan.matvec(th, xt)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("seed", range(10))
def test_random_models(seed):
    rng = np.random.default_rng(1000 + seed)
    herm = seed % 3 != 0
    m = W.random_model(rng, n_sites=int(rng.integers(1, 7)), max_dim=20000, hermitian=herm,
                       n_params=int(rng.integers(1, 5)))
    print(f"random model seed={seed} D={m.dim} terms={len(m.terms)}", flush=True)
    p = Plan(m, require_hermitian=herm)
    x = W.random_state(m.dim, rng)
    assert rel_err(gpu_matvec(p, m.theta, x), mf.matvec(m, x)) <= TOL_Z
    x32 = x.astype(np.complex64)
    y32 = gpu_matvec(p, m.theta, x32)
    assert rel_err(y32, mf.matvec(m, x32.astype(np.complex128))) <= TOL_C


@pytest.mark.parametrize("seed", range(4))
def test_debug_sources_bit_exact(seed):
    rng = np.random.default_rng(2000 + seed)
    m = W.random_model(rng, n_sites=5, max_dim=6000)
    p = Plan(m)
    got = p.debug_sources(0, m.dim).cpu().numpy()
    ref = mf.sources(m, 0, m.dim)[:, p.offdiag_terms()]
    assert np.array_equal(got, ref)


def test_debug_sources_config2_window():
    m, _ = W.config(2, with_state=False)
    p = Plan(m)
    for F0 in (0, m.dim // 3 + 17, m.dim - 5000):
        got = p.debug_sources(F0, 5000).cpu().numpy()
        ref = mf.sources(m, F0, 5000)[:, p.offdiag_terms()]
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("k", [1, 5])
def test_small_configs_full(k):
    m, x = W.config(k)
    p = Plan(m)
    assert rel_err(gpu_matvec(p, m.theta, x), mf.matvec(m, x)) <= TOL_Z


def sample_rows(D, rng, n=3000):
    rows = np.concatenate([np.arange(min(256, D)), np.arange(max(0, D - 256), D),
                           rng.choice(D, size=min(n, D), replace=False)])
    return np.unique(rows).astype(np.int64)


def test_config2_full_size_sampled():
    """Ferrimagnetic ring, D = 60,466,176, c128, default kernel choice: sampled rows (both ends and a
    random sample) against the oracle.  The whole vector and the sum rule sum_F (H x)_F = <H 1|x> are
    checked with the benchmark's kernel shape in test_gpu_fullsize.py."""
    m, x = W.config(2)
    p = Plan(m)
    y = gpu_matvec(p, m.theta, x)
    rows = sample_rows(m.dim, np.random.default_rng(0))
    ref = mf.matvec(m, x, rows=rows)
    assert rel_err(y[rows], ref) <= TOL_Z
    assert np.all(np.isfinite(y))


def test_config3_full_size_sampled_c64():
    """Spin-1 4x4 torus, D = 43,046,721, c64 kernel against the FP64 oracle on sampled rows."""
    m, x = W.config(3)
    p = Plan(m)
    y = gpu_matvec(p, m.theta, x)
    rows = sample_rows(m.dim, np.random.default_rng(1))
    ref = mf.matvec(m, x.astype(np.complex128), rows=rows)
    assert rel_err(y[rows], ref) <= TOL_C


def test_edge_cases():
    # no terms: y = 0 exactly
    m = Model([spin_site(2), boson_site(3)], [], np.ones(1))
    x = W.random_state(m.dim, np.random.default_rng(0))
    assert np.all(gpu_matvec(Plan(m), m.theta, x) == 0)
    # one site, one raise/lower pair, ragged D (not a multiple of the block)
    m = Model([spin_site(5)], [Term(0, OP_RAISE, -1, OP_Z, 0, 0.3), Term(0, OP_LOWER, -1, OP_Z, 0, 0.3)],
              np.ones(1))
    x = W.random_state(m.dim, np.random.default_rng(1))
    assert rel_err(gpu_matvec(Plan(m), m.theta, x), mf.matvec(m, x)) <= TOL_Z
    m = W.ferrimagnetic_ring(9)       # D = 2^5 3^4 = 2592: several blocks and a ragged tail
    x = W.random_state(m.dim, np.random.default_rng(2))
    assert rel_err(gpu_matvec(Plan(m), m.theta, x), mf.matvec(m, x)) <= TOL_Z


def test_argument_errors():
    from paper_2606_02169_amd import _lib as L
    m, x = W.config(1)
    p = Plan(m)
    xt = torch.from_numpy(x).cuda()
    th = torch.as_tensor(m.theta, device="cuda")
    import ctypes
    st = L.lib().mrmf_matvec_z(p.handle, ctypes.c_void_p(p.ws.data_ptr()), ctypes.c_void_p(th.data_ptr()),
                               ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(xt.data_ptr()), None)
    assert st == L.MRMF_E_INVALID_ARG        # in place: the gather reads x while writing y
    with pytest.raises(ValueError):
        p.matvec(th, xt[:100])
