"""The paper's chain testbeds (spin-1 ring N=15, D = 3^15; mixed ring (1/2)^6 (1)^6 (3/2)^6, D = 24^6) on
the GPU: sampled rows against the oracle, and the same structure at oracle size through Lanczos."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lanczos as olz
from oracle import mf
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_paper_testbed_matvec_sampled(which):
    from paper_2606_02169_amd.plan import Plan
    m = W.paper_c1() if which == "c1" else W.paper_c2()
    rng = np.random.default_rng(21)
    x = W.random_state(m.dim, rng)
    p = Plan.from_model(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device=DEV)
    xt = torch.from_numpy(x).to(DEV)
    p.autotune(th, xt)
    y = p.matvec(th, xt)
    torch.cuda.synchronize()
    print(m.name, m.dim, p.kernel_info(), flush=True)
    rows = np.unique(np.concatenate([np.arange(200), np.arange(m.dim - 200, m.dim),
                                     rng.choice(m.dim, 3000, replace=False)])).astype(np.int64)
    got = y[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    assert rel_err(got, mf.matvec(m, x, rows=rows)) <= 1e-12


def test_staggered_ring_lanczos_small():
    """The same structure (spin-1 ring, staggered field) at N = 8 against the oracle's Lanczos."""
    from paper_2606_02169_amd.plan import Plan
    m = W.staggered_xxz_ring([2] * 8)
    x = W.random_state(m.dim, np.random.default_rng(3))
    p = Plan.from_model(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device=DEV)
    r = p.lanczos(th, torch.from_numpy(x).to(DEV), 60)["result"].cpu().numpy()
    o = olz.lanczos(lambda v: mf.matvec(m, v), x, 60)
    assert abs(r[0] - o["theta"]) <= 1e-10 * abs(o["theta"])
