"""GPU Lanczos (mrmf_lanczos) against the oracle's Lanczos (same algorithm, same start vector) and
against closed forms.  Energies and residuals are compared, never eigenvectors."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lanczos as olz
from oracle import mf

pytestmark = pytest.mark.gpu


def Plan(model):
    from paper_2606_02169_amd.plan import Plan as P
    return P.from_model(model)


def run(model, x, m, **kw):
    p = Plan(model)
    th = torch.as_tensor(model.theta, dtype=torch.float64, device="cuda")
    out = p.lanczos(th, torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda(), m, **kw)
    torch.cuda.synchronize()
    res = out["result"].cpu().numpy()
    k = int(res[3]) if np.isfinite(res[3]) else 0
    return dict(theta=res[0], resid_est=res[1], resid=res[2], steps=k,
                alpha=out["alpha"].cpu().numpy()[:k], beta=out["beta"].cpu().numpy()[:k], u=out["u"])


def test_config1_against_oracle_lanczos():
    m, x = W.config(1)
    g = run(m, x, 50)
    o = olz.lanczos(lambda v: mf.matvec(m, v), x, 50)
    print(f"theta gpu={g['theta']!r} oracle={o['theta']!r} resid {g['resid']:.3e} / {o['resid']:.3e}")
    assert g["steps"] == o["steps"] == 50
    assert abs(g["theta"] - o["theta"]) <= 1e-12 * abs(o["theta"])
    assert np.max(np.abs(g["alpha"][:20] - o["alpha"][:20])) < 1e-11
    assert np.max(np.abs(g["beta"][:20] - o["beta"][:20])) < 1e-11
    assert g["resid"] < 1e-8 and abs(g["resid_est"] - g["resid"]) < 1e-8
    ev = np.linalg.eigvalsh(__import__("oracle.kron", fromlist=["x"]).sparse_H(m).toarray())[0]
    assert abs(g["theta"] - ev) <= g["resid"] + 1e-12          # Weyl bound


def test_ferrimagnetic_ring_reduced_against_oracle():
    m, x = W.config(2, reduced=12)                          # D = 2^6 3^6 = 46656
    g = run(m, x, 60)
    o = olz.lanczos(lambda v: mf.matvec(m, v), x, 60)
    print(f"theta gpu={g['theta']!r} oracle={o['theta']!r}")
    assert abs(g["theta"] - o["theta"]) <= 1e-12 * abs(o["theta"])
    assert abs(g["resid"] - o["resid"]) <= 1e-3 * o["resid"] + 1e-12


def test_no_reorth_recurrence():
    m, x = W.config(2, reduced=10)
    g = run(m, x, 40, reorth="none")
    o = olz.lanczos(lambda v: mf.matvec(m, v), x, 40, reorth=False)
    assert np.max(np.abs(g["alpha"][:15] - o["alpha"][:15])) < 1e-10
    assert abs(g["theta"] - o["theta"]) <= 1e-10 * abs(o["theta"])


def test_fp32_form_energy_error():
    """c64 matvec inside the FP64 recurrence: ground energy against the FP64 oracle within 1e-5."""
    m, x = W.config(3, reduced=3)                           # spin-1 3x3 torus, D = 19683
    p = Plan(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device="cuda")
    x128 = x.astype(np.complex128)
    out = p.lanczos(th, torch.from_numpy(x128).cuda(), 80, precision="c_in_z")
    torch.cuda.synchronize()
    theta32 = float(out["result"][0])
    o = olz.lanczos(lambda v: mf.matvec(m, v), x128, 80)
    err = abs(theta32 - o["theta"]) / abs(o["theta"])
    print(f"fp32-form theta {theta32!r} fp64 oracle {o['theta']!r} rel err {err:.2e}")
    assert err <= 1e-5


def test_breakdown_on_eigenvector():
    m = W.ferrimagnetic_ring(8)
    x = np.zeros(m.dim, dtype=np.complex128)
    x[-1] = 1.0                                             # fully polarised: an eigenvector
    g = run(m, x, 10)
    assert g["steps"] == 1
    assert abs(g["theta"] - mf.matvec(m, x)[-1].real) < 1e-14


def test_zero_start_vector():
    m = W.ferrimagnetic_ring(6)
    g = run(m, np.zeros(m.dim, dtype=np.complex128), 5)
    assert g["steps"] == 0 and np.isnan(g["theta"])


@pytest.mark.parametrize("reorth", ["cgs2_cond", "partial"])
def test_breakdown_and_zero_start_other_reorth(reorth):
    """The conditional and partial forms stop like the full one: an eigenvector start breaks down after one
    step with its exact energy, a zero start takes no step."""
    m = W.ferrimagnetic_ring(8)
    x = np.zeros(m.dim, dtype=np.complex128)
    x[-1] = 1.0
    g = run(m, x, 10, reorth=reorth)
    assert g["steps"] == 1
    assert abs(g["theta"] - mf.matvec(m, x)[-1].real) < 1e-14
    z = run(m, np.zeros(m.dim, dtype=np.complex128), 5, reorth=reorth)
    assert z["steps"] == 0 and np.isnan(z["theta"])


@pytest.mark.parametrize("reorth", ["cgs2", "cgs2_cond", "partial"])
def test_krylov_space_exhausted(reorth):
    """More steps than the dimension (ferrimagnetic ring N = 4, D = 36, 80 steps): the recurrence breaks
    down once the Krylov space is exhausted (a basis of at most D vectors), and the Ritz value is the
    lowest eigenvalue of the oracle's dense H to rounding."""
    m = W.ferrimagnetic_ring(4)
    x = W.random_state(m.dim, np.random.default_rng(21))
    g = run(m, x, 80, reorth=reorth)
    ev = np.linalg.eigvalsh(__import__("oracle.kron", fromlist=["x"]).dense_H(m))[0]
    print(f"{reorth}: steps {g['steps']} theta {g['theta']!r} exact {ev!r} residual {g['resid']:.2e}", flush=True)
    assert 1 <= g["steps"] <= m.dim
    assert abs(g["theta"] - ev) <= 1e-12 * abs(ev)
    assert g["resid"] <= 1e-10


def test_free_fermion_closed_form_large():
    """XX chain N=20 in a field (D = 2^20): E0 = sum_{eps_k<0} eps_k - N h/2, no oracle involved."""
    N, J, h = 20, 1.0, 0.25
    m = W.xx_chain_in_field(N, J, h)
    eps = J * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)) + h
    e0 = eps[eps < 0].sum() - N * h / 2
    x = W.random_state(m.dim, np.random.default_rng(9))
    g = run(m, x, 160)
    print(f"E0 closed form {e0!r} gpu {g['theta']!r} resid {g['resid']:.2e}")
    assert abs(g["theta"] - e0) <= max(g["resid"], 1e-11)
    assert abs(g["theta"] - e0) < 1e-9


def test_long_run_orthonormal_basis():
    """240 steps on config 1 (D = 4096): the whole basis stays orthonormal to rounding, the first steps agree
    with the oracle's recurrence (later alpha_j of any two codes part once the ground state has converged),
    and the Ritz value with the oracle's."""
    m, x = W.config(1)
    p = Plan(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device="cuda")
    out = p.lanczos(th, torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda(), 240,
                    keep_basis=True)
    torch.cuda.synchronize()
    res = out["result"].cpu().numpy()
    o = olz.lanczos(lambda v: mf.matvec(m, v), x, 240)
    assert int(res[3]) == o["steps"] == 240
    assert abs(res[0] - o["theta"]) <= 1e-12 * abs(o["theta"])
    a = out["alpha"].cpu().numpy()
    assert np.max(np.abs(a[:30] - o["alpha"][:30])) < 1e-12
    V = out["V"].reshape(241, -1)[:240].cpu().numpy()
    G = V.conj() @ V.T
    assert np.max(np.abs(G - np.eye(240))) <= 1e-12


@pytest.mark.parametrize("m_steps", [50, 240])
def test_conditional_second_pass(m_steps):
    """Gram-Schmidt with the second pass only where the first one shrank ||w|| by more than 1/sqrt(2):
    config 1 against the oracle's CGS2 recurrence (the same Krylov basis up to rounding), and the whole
    basis orthonormal to rounding, also over 240 steps past the lowest eigenvalues' convergence."""
    m, x = W.config(1)
    p = Plan(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device="cuda")
    out = p.lanczos(th, torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda(), m_steps,
                    reorth="cgs2_cond", keep_basis=True)
    torch.cuda.synchronize()
    res = out["result"].cpu().numpy()
    o = olz.lanczos(lambda v: mf.matvec(m, v), x, m_steps)
    assert int(res[3]) == o["steps"] == m_steps
    assert abs(res[0] - o["theta"]) <= 1e-12 * abs(o["theta"])
    a = out["alpha"].cpu().numpy()
    assert np.max(np.abs(a[:20] - o["alpha"][:20])) < 1e-11
    V = out["V"].reshape(m_steps + 1, -1)[:m_steps].cpu().numpy()
    assert np.max(np.abs(V.conj() @ V.T - np.eye(m_steps))) <= 1e-12
    assert res[2] < 1e-8


def _basis(model, x, m_steps, reorth):
    p = Plan(model)
    th = torch.as_tensor(model.theta, dtype=torch.float64, device="cuda")
    out = p.lanczos(th, torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda(), m_steps,
                    reorth=reorth, keep_basis=True)
    torch.cuda.synchronize()
    res = out["result"].cpu().numpy()
    k = int(res[3])
    V = out["V"].reshape(m_steps + 1, -1)[:k].cpu().numpy()
    loss = float(np.max(np.abs(V.conj() @ V.T - np.eye(k))))
    return res, out["counts"].cpu().numpy(), loss


@pytest.mark.parametrize("m_steps", [50, 240])
def test_partial_reorthogonalisation(m_steps):
    """Simon's partial reorthogonalisation on config 1: the Ritz value of the oracle's fully
    reorthogonalised recurrence to 1e-12, a semi-orthogonal basis (every |<v_i|v_k>| near sqrt(eps) at
    most) while the plain recurrence loses orthogonality on the same run, and Gram-Schmidt passes at a
    minority of the steps."""
    m, x = W.config(1)
    res, counts, loss = _basis(m, x, m_steps, "partial")
    o = olz.lanczos(lambda v: mf.matvec(m, v), x, m_steps)
    _, _, loss_none = _basis(m, x, m_steps, "none")
    print(f"m={m_steps} theta {res[0]!r} oracle {o['theta']!r} passes {counts[1]} of {int(res[3])} steps, "
          f"max |V^H V - I| {loss:.2e} (no reorthogonalisation: {loss_none:.2e})", flush=True)
    assert int(res[3]) == o["steps"] == m_steps
    assert abs(res[0] - o["theta"]) <= 1e-12 * abs(o["theta"])
    assert loss <= 1e-7
    assert res[2] < 1e-8
    if m_steps == 240:
        assert loss_none > 1e-3          # the plain recurrence does lose orthogonality here
        assert 0 < counts[1] < m_steps // 2
    else:
        assert counts[1] < m_steps // 2


def test_partial_reorthogonalisation_free_fermions():
    """Partial reorthogonalisation on the XX chain N = 20 in a field (D = 2^20) against the closed form."""
    N, J, h = 20, 1.0, 0.25
    m = W.xx_chain_in_field(N, J, h)
    eps = J * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)) + h
    e0 = eps[eps < 0].sum() - N * h / 2
    x = W.random_state(m.dim, np.random.default_rng(9))
    p = Plan(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device="cuda")
    out = p.lanczos(th, torch.from_numpy(x).cuda(), 160, reorth="partial")
    torch.cuda.synchronize()
    res, counts = out["result"].cpu().numpy(), out["counts"].cpu().numpy()
    print(f"E0 closed form {e0!r} gpu {res[0]!r} resid {res[2]:.2e}, passes {counts[1]}", flush=True)
    assert abs(res[0] - e0) <= max(res[2], 1e-11)
    assert abs(res[0] - e0) < 1e-9


def test_partial_reorthogonalisation_fp32_form():
    """Partial reorthogonalisation with the c64 matvec inside the FP64 recurrence on the 12-site reduced
    ferrimagnetic ring (D = 46656), 150 steps: the estimate takes FP32's epsilon, so the basis stays
    semi-orthogonal to about sqrt(eps32) and the Ritz value stays within 1e-5 of the oracle's fully
    reorthogonalised FP64 value, and not below it by more than FP32 rounding (no spurious level)."""
    m, x = W.config(2, reduced=12)
    p = Plan(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device="cuda")
    out = p.lanczos(th, torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda(), 150,
                    precision="c_in_z", reorth="partial", keep_basis=True)
    torch.cuda.synchronize()
    res, counts = out["result"].cpu().numpy(), out["counts"].cpu().numpy()
    k = int(res[3])
    V = out["V"].reshape(151, -1)[:k].cpu().numpy()
    loss = float(np.max(np.abs(V.conj() @ V.T - np.eye(k))))
    o = olz.lanczos(lambda v: mf.matvec(m, v), x, 150)
    rel = (res[0] - o["theta"]) / abs(o["theta"])
    print(f"fp32 form, partial: theta {res[0]!r} oracle fp64 {o['theta']!r} rel {rel:.2e} passes {counts[1]} "
          f"of {k}, max |V^H V - I| {loss:.2e}, residual {res[2]:.2e}", flush=True)
    assert k == 150
    assert abs(rel) <= 1e-5
    assert rel >= -1e-6
    assert loss <= 2e-3


def simon_passes(alpha, beta, D, eps):
    """Gram-Schmidt passes that partial reorthogonalisation prescribes for a run with these alpha, beta:
    Simon's recurrence for the estimates omega_{j+1,k} of <v_{j+1}|v_k>, a rounding term 2 eps ||T|| of
    the sign that increases |omega|, omega_{j+1,j} = eps64 sqrt(D) ||T|| / beta_j, a pass where an estimate
    exceeds sqrt(eps) and at the step after, the estimates restarting at eps64 sqrt(D) after a pass
    (||T|| is the running Gershgorin estimate max |alpha_i| + beta_i + beta_{i-1})."""
    eps64 = np.finfo(np.float64).eps
    level = eps64 * np.sqrt(D)
    rows = {0: np.zeros(0)}
    tnorm, force, passes = 0.0, False, 0
    for j in range(len(alpha)):
        a, b = alpha, beta
        tn = max(tnorm, abs(a[j]) + b[j] + (b[j - 1] if j > 0 else 0.0))
        cur = np.append(rows[j], 1.0)                                   # omega_{j,k}, k <= j
        prev = np.append(rows[j - 1], 1.0) if j > 0 else None           # omega_{j-1,k}, k <= j-1
        new = np.empty(j + 1)
        for k in range(j):
            t = b[k] * cur[k + 1] + (a[k] - a[j]) * cur[k]
            if k > 0:
                t += b[k - 1] * cur[k - 1]
            if j > 0:
                t -= b[j - 1] * prev[k]
            t += (2.0 if t >= 0 else -2.0) * eps * tn
            new[k] = t / b[j]
        new[j] = level * tn / b[j]
        over = np.max(np.abs(new)) > np.sqrt(eps)
        if over or force:
            passes += 1
            new[:] = level
        force = over
        rows[j + 1] = new
        tnorm = max(tnorm, abs(a[j]) + b[j] + (b[j - 1] if j > 0 else 0.0))
    return passes


@pytest.mark.parametrize("prec", ["z", "c_in_z"])
def test_partial_reorthogonalisation_pass_count(prec):
    """The passes the device took equal those Simon's recurrence prescribes for the run's own alpha and beta
    (the estimate replayed on the host from the method's definition): config 1, 240 steps, both forms."""
    m, x = W.config(1)
    p = Plan(m)
    th = torch.as_tensor(m.theta, dtype=torch.float64, device="cuda")
    out = p.lanczos(th, torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda(), 240,
                    precision=prec, reorth="partial")
    torch.cuda.synchronize()
    k = int(out["result"][3])
    a, b = out["alpha"].cpu().numpy()[:k], out["beta"].cpu().numpy()[:k]
    eps = np.finfo(np.float32).eps if prec == "c_in_z" else np.finfo(np.float64).eps
    want = simon_passes(a, b, m.dim, float(eps))
    got = int(out["counts"].cpu().numpy()[1])
    print(f"{prec}: passes device {got} host replay {want} in {k} steps", flush=True)
    assert k == 240 and got == want and got > 0


def test_lanczos_graph_replays_match_eager():
    """The 12-site Heisenberg chain (D = 4096, where every kernel is launch-bound): one 50-step mrmf_lanczos
    call captured in a HIP graph and replayed three times, with eager Lanczos runs on other start vectors
    and synchronisations between the replays; each replay's alpha, beta and result equal the eager call's
    bitwise (the outputs are cleared before each replay, so a replay that did nothing would fail)."""
    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    m, x = W.config(1)
    p = Plan(m)
    th, xt = t(m.theta), t(x)
    ref = p.lanczos(th, xt, 50)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = p.lanczos(th, xt, 50)
    rng = np.random.default_rng(9100)
    for k in range(3):
        out["alpha"].zero_()
        out["beta"].zero_()
        out["result"].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        other = p.lanczos(th, t(W.random_state(m.dim, rng)), 20)
        torch.cuda.synchronize()
        print(k, float(out["result"][0]), float(ref["result"][0]), flush=True)
        assert torch.equal(out["alpha"], ref["alpha"]) and torch.equal(out["beta"], ref["beta"])
        assert torch.equal(out["result"], ref["result"])
        assert torch.isfinite(other["result"][0])
