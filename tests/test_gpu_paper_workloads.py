"""The paper's chain testbeds (spin-1 ring N=15, D = 3^15; mixed ring (1/2)^6 (1)^6 (3/2)^6, D = 24^6) on
the GPU: the whole output vector (C1, C2) and sampled rows (C2) against the oracle, C2's Lanczos residual
recomputed by the oracle, and the same structure at oracle size through Lanczos."""
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
    if which == "c1":   # D = 14,348,907: the whole vector (C2's is checked whole below)
        assert rel_err(y.cpu().numpy(), mf.matvec(m, x)) <= 1e-12
        return
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


def test_paper_c2_whole_vector_and_certified_lanczos():
    """The mixed ring (1/2)^6 (1)^6 (3/2)^6 at full size (D = 191,102,976; 3.06 GB per c128 vector, the
    64-bit-addressing form of the generated kernel): every element of y = H x against the oracle, then 60
    Lanczos steps with partial reorthogonalisation whose Ritz vector's residual the oracle recomputes
    (it must equal the GPU's, and it bounds the distance of the FP64 energy to the spectrum)."""
    from paper_2606_02169_amd.plan import Plan
    m = W.paper_c2()
    x = W.random_state(m.dim, np.random.default_rng(22))
    p = Plan.from_model(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device=DEV)
    xt = torch.from_numpy(x).to(DEV)
    p.autotune(th, xt)
    y = p.matvec(th, xt).cpu().numpy()
    del xt
    torch.cuda.empty_cache()
    ref = mf.matvec(m, x)
    e = rel_err(y, ref)
    worst, bound = float(np.max(np.abs(y - ref))), 1e-12 * float(np.max(np.abs(ref)))
    print(f"C2 whole vector: rel 2-norm err {e:.2e}, max |err| {worst:.2e} (bound {bound:.2e})", flush=True)
    del y, ref
    assert e <= 1e-12 and worst <= bound
    r = p.lanczos(th, torch.from_numpy(x).to(DEV), 60, reorth="partial")
    res = r["result"].cpu().numpy()
    u = r["u"].cpu().numpy()
    del r
    torch.cuda.empty_cache()
    theta, r_gpu = float(res[0]), float(res[2])
    r_oracle = float(np.linalg.norm(mf.matvec(m, u) - theta * u))
    print(f"C2 Lanczos: theta {theta!r} residual gpu {r_gpu:.4e} oracle {r_oracle:.4e}", flush=True)
    assert int(res[3]) == 60 and abs(np.linalg.norm(u) - 1.0) <= 1e-10
    assert abs(r_gpu - r_oracle) <= 1e-10 * r_oracle + 1e-13 * abs(theta)
