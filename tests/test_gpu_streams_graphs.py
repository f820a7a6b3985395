"""The plain matvec and the propagation step on non-default streams and inside captured HIP graphs:
replays (with eager work and synchronisation between them) against the eager result, and two plans
running on two streams at once."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import mf
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def mk(model):
    from paper_2606_02169_amd.plan import Plan
    return Plan.from_model(model)


@pytest.mark.parametrize("kind", ["specialized", "generic"])
def test_matvec_graph_replays(kind):
    m, x = W.config(2, reduced=12)
    p = mk(m)
    p.set_kernel(kind)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device=DEV)
    xt = torch.from_numpy(x).to(DEV)
    y = torch.empty_like(xt)
    z = torch.empty_like(xt)
    p.prepare(torch.complex128)            # compile before capture
    eager = p.matvec(th, p.matvec(th, xt)).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p.matvec(th, xt, out=y)            # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.matvec(th, xt, out=y)
        p.matvec(th, y, out=z)
    for k in range(4):
        xt.mul_(1.0)                        # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(z, eager), k
    assert rel_err(z.cpu().numpy(), mf.matvec(m, mf.matvec(m, x))) <= 1e-12


def test_two_plans_two_streams():
    m1, x1 = W.config(2, reduced=12)
    m2 = W.staggered_xxz_ring([2] * 10)
    x2 = W.random_state(m2.dim, np.random.default_rng(9))
    p1, p2 = mk(m1), mk(m2)
    t1 = torch.as_tensor(m1.theta, dtype=torch.float64, device=DEV)
    t2 = torch.as_tensor(m2.theta, dtype=torch.float64, device=DEV)
    a, b = torch.from_numpy(x1).to(DEV), torch.from_numpy(x2).to(DEV)
    ref1, ref2 = p1.matvec(t1, a).clone(), p2.matvec(t2, b).clone()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        ya = [p1.matvec(t1, a) for _ in range(5)]
    with torch.cuda.stream(s2):
        yb = [p2.matvec(t2, b) for _ in range(5)]
    torch.cuda.synchronize()
    for u in ya:
        assert torch.equal(u, ref1)
    for v in yb:
        assert torch.equal(v, ref2)


def test_fused_propagation_step_in_graph():
    """One fused Chebyshev-step launch captured and replayed: the same numbers as the eager propagate."""
    m, x = W.config(2, reduced=12)
    p = mk(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device=DEV)
    xt = torch.from_numpy(x).to(DEV)
    bnd = p.norm_bound(m.theta)
    eager = p.propagate(th, xt, 0.1, 2, bounds=(-bnd, bnd))["x"].clone()
    out = torch.empty_like(xt)
    p.propagate(th, xt, 0.1, 2, bounds=(-bnd, bnd), out=out)         # compiles the kernel, warms up
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    keep = {}
    with torch.cuda.stream(s):
        keep["warm"] = p.propagate(th, xt, 0.1, 2, bounds=(-bnd, bnd), out=out)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        keep["cap"] = p.propagate(th, xt, 0.1, 2, bounds=(-bnd, bnd), out=out)
    for k in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
