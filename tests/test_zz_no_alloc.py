"""mrmf_adjoint_z_noalloc (the adjoint with its scratch in a static device array, for callers that cannot
allocate) against mrmf_adjoint_z through the C ABI: calls in a row, the second on a smaller input, each
output equal to the existing entry point's."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def raw_adjoint(p, th, x, g, noalloc):
    from paper_2606_02169_amd import _lib as L
    from paper_2606_02169_amd.plan import _ptr, _stream
    gx = torch.full_like(x, float("nan"))
    gt = torch.full((max(1, p.n_params),), float("nan"), dtype=torch.float64, device=DEV)
    if noalloc:
        st = L.lib().mrmf_adjoint_z_noalloc(p.handle, _ptr(p.ws), _ptr(th), _ptr(x), _ptr(g), _ptr(gx), _ptr(gt),
                                            _stream(DEV))
    else:
        nb = ctypes.c_size_t()
        L.call("mrmf_adjoint_scratch_bytes", p.handle, ctypes.byref(nb))
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=DEV)
        st = L.lib().mrmf_adjoint_z(p.handle, _ptr(p.ws), _ptr(th), _ptr(x), _ptr(g), _ptr(gx), _ptr(gt),
                                    _ptr(scratch), nb.value, _stream(DEV))
    assert st == L.MRMF_OK, L.status_string(st)
    torch.cuda.synchronize()
    return gx.cpu().numpy(), gt.cpu().numpy()[: p.n_params]


def case(model, seed, generic):
    from paper_2606_02169_amd.plan import Plan
    p = Plan.from_model(model, device=DEV)
    if generic:
        p.set_kernel("generic")
    else:
        assert p.grad_kernel_ready()          # build the generated kernel first: the no-alloc call compiles nothing
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(W.random_state(model.dim, rng)).to(DEV)
    g = torch.from_numpy(W.random_state(model.dim, rng)).to(DEV)
    th = torch.as_tensor(model.theta, dtype=torch.float64, device=DEV)
    return p, th, x, g


def check(p, th, x, g, label):
    gx0, gt0 = raw_adjoint(p, th, x, g, noalloc=False)
    gx1, gt1 = raw_adjoint(p, th, x, g, noalloc=True)
    print(f"{label}: D={p.D} params={p.n_params} grad_x rel err {rel_err(gx1, gx0):.2e} "
          f"grad_theta max abs diff {np.max(np.abs(gt1 - gt0)) if gt0.size else 0.0:.2e}", flush=True)
    assert np.all(np.isfinite(gx1)) and np.all(np.isfinite(gt1))
    assert rel_err(gx1, gx0) <= 1e-12
    assert rel_err(gt1, gt0) <= 1e-12
    # same kernels and the same fixed-order reductions: identical bits
    assert np.array_equal(gx1, gx0) and np.array_equal(gt1, gt0)


def test_noalloc_adjoint_two_calls_second_smaller():
    big, _ = W.config(5)                                  # Tavis-Cummings, D = 266,240, 25 couplings
    small, _ = W.config(2, reduced=8)                     # ring of 8 sites, D = 1296, 4 couplings
    pb = case(big, 1, generic=False)
    ps = case(small, 2, generic=False)
    check(*pb, "first call (generated kernel)")
    check(*ps, "second call, smaller input")
    pg = case(small, 3, generic=True)
    check(*pg, "third call, generic pass")
