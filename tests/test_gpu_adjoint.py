"""The hand-written adjoint (mrmf_adjoint_z behind MatvecFn) against the oracle's gradient formulas,
central finite differences of the GPU loss, and torch.autograd.gradcheck; both forms (the plan's matvec
plus the generated coupling-gradient kernel, and the generic fused gather pass)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import grad as ograd
from oracle import mf
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def mk(model, **kw):
    from paper_2606_02169_amd.plan import Plan
    return Plan.from_model(model, **kw)


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("kind", ["auto", "generic"])
@pytest.mark.parametrize("seed", range(8))
def test_adjoint_random_models(seed, kind):
    rng = np.random.default_rng(9000 + seed)
    m = W.random_model(rng, n_sites=int(rng.integers(2, 6)), max_dim=6000, n_params=int(rng.integers(1, 40)),
                       n_terms=int(rng.integers(4, 40)))
    print(f"seed={seed} kind={kind} D={m.dim} params={m.n_params} terms={len(m.terms)}", flush=True)
    x = W.random_state(m.dim, rng)
    g = W.random_state(m.dim, rng)
    p = mk(m)
    if kind == "generic":
        p.set_kernel("generic")
    else:
        assert p.grad_kernel_ready()
    gx, gt = p.adjoint(t(m.theta), t(x), t(g))
    rgx, rgt = ograd.adjoint(m, x, g)
    assert rel_err(gx.cpu().numpy(), rgx) <= 1e-12
    assert np.max(np.abs(gt.cpu().numpy() - rgt)) <= 1e-12 * max(1.0, np.max(np.abs(rgt)))


def loss_torch(p, theta, x):
    from paper_2606_02169_amd.plan import MatvecFn
    y = MatvecFn.apply(p, theta, x)
    return torch.vdot(x, y).real / torch.vdot(x, x).real


def test_tavis_cummings_rayleigh_gradients():
    """Config: 12 spin-1/2 + boson cut at 64, L = Re<x|H|x>/<x|x>; autograd through MatvecFn against
    the Hellmann-Feynman closed forms and central finite differences in FP64."""
    m, x = W.config(5)
    p = mk(m)
    assert p.grad_kernel_ready()
    theta = t(m.theta).requires_grad_(True)
    xt = t(x).requires_grad_(True)
    L = loss_torch(p, theta, xt)
    L.backward()
    L_ref, gx_ref, gt_ref = ograd.rayleigh(m, x)
    assert abs(L.item() - L_ref) <= 1e-13 * max(1.0, abs(L_ref))
    assert rel_err(xt.grad.cpu().numpy(), gx_ref) <= 1e-11
    assert np.max(np.abs(theta.grad.cpu().numpy() - gt_ref)) <= 1e-12
    # central differences of the GPU loss: every coupling, and three random directions in x
    def Lval(th, xx):
        with torch.no_grad():
            return loss_torch(p, th, xx).item()
    h = 1e-5
    gt = theta.grad.cpu().numpy()
    th0 = t(m.theta)
    for q in range(m.n_params):
        e = torch.zeros_like(th0)
        e[q] = h
        fd = (Lval(th0 + e, t(x)) - Lval(th0 - e, t(x))) / (2 * h)
        assert abs(fd - gt[q]) <= 1e-9, (q, fd, gt[q])
    rng = np.random.default_rng(55)
    gxv = xt.grad.cpu().numpy()
    for _ in range(3):
        d = W.random_state(m.dim, rng)
        fd = (Lval(th0, t(x + h * d)) - Lval(th0, t(x - h * d))) / (2 * h)
        # directional derivative of a real loss along d: Re <grad_x | d>
        assert abs(fd - np.vdot(gxv, d).real) <= 1e-8, fd


def test_gradcheck_tiny():
    rng = np.random.default_rng(4)
    m = W.random_model(rng, n_sites=3, max_dim=40, n_params=3, n_terms=10)
    p = mk(m)
    theta = t(m.theta).requires_grad_(True)
    x = t(W.random_state(m.dim, rng)).requires_grad_(True)
    from paper_2606_02169_amd.plan import MatvecFn
    assert torch.autograd.gradcheck(lambda th, xx: MatvecFn.apply(p, th, xx), (theta, x), eps=1e-6,
                                    atol=1e-8, rtol=1e-6)


def test_adjoint_rejects_non_hermitian():
    from paper_2606_02169_amd import _lib as L
    rng = np.random.default_rng(1)
    m = W.random_model(rng, n_sites=3, max_dim=100, hermitian=False)
    p = mk(m, require_hermitian=False)
    x = t(W.random_state(m.dim, rng))
    with pytest.raises(L.MrmfError) as e:
        p.adjoint(t(m.theta), x, x.clone())
    assert e.value.status == L.MRMF_E_NOT_HERMITIAN


@pytest.mark.parametrize("n_params,bpc", [(60, 0), (48, 8), (7, 1)])
def test_adjoint_parameter_counts(n_params, bpc):
    """Beyond 48 parameters the generic pass runs; at the limit and below, the generated kernel with eight
    blocks per CU and with one (D = 82,944 on 256 blocks: a ragged second row per thread)."""
    rng = np.random.default_rng(9100 + n_params)
    m = W.random_model(rng, n_sites=10, max_dim=500000, n_params=n_params, n_terms=70)
    x, g = W.random_state(m.dim, rng), W.random_state(m.dim, rng)
    p = mk(m)
    p.set_tuning(grad_blocks_per_cu=bpc)
    assert p.grad_kernel_ready() == (n_params <= 48)
    print(f"D={m.dim} params={m.n_params} terms={len(m.terms)} bpc={bpc}", flush=True)
    gx, gt = p.adjoint(t(m.theta), t(x), t(g))
    rgx, rgt = ograd.adjoint(m, x, g)
    assert rel_err(gx.cpu().numpy(), rgx) <= 1e-12
    assert np.max(np.abs(gt.cpu().numpy() - rgt)) <= 1e-12 * max(1.0, np.max(np.abs(rgt)))
    gx2, gt2 = p.adjoint(t(m.theta), t(x), t(g))                       # deterministic: same bits again
    assert torch.equal(gx, gx2) and torch.equal(gt, gt2)
