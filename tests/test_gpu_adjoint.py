"""GPU KKT adjoint (through the C-ABI) against the float64 reference
gradient of the oracle and against exact invariants."""
import numpy as np
import pytest

import oracle
from oracle.adjoint import gradients
from oracle.problem import account
from workloads import make_config

pytestmark = pytest.mark.gpu


def _gpu_adjoint(uni, book, C, **settings):
    import torch
    from paper_2606_23367_amd.solver import Solver, to_device
    P = to_device(uni, book)
    s = Solver(0)
    out = s.solve(P, **settings)
    dmu, dB = s.adjoint(torch.as_tensor(C, device="cuda:0"))
    torch.cuda.synchronize()
    return ({k: v.cpu().numpy() for k, v in out.items()}, dmu.cpu().numpy(),
            dB.cpu().numpy())


@pytest.mark.parametrize("gamma", [1000.0, 1.0])
def test_adjoint_matches_reference(gamma):
    uni, book = make_config("c4", 0, N=800, M=6, k=10, gamma=gamma)
    rng = np.random.default_rng(0)
    C = rng.normal(size=(book.m, uni.n))
    host, dmu, dB = _gpu_adjoint(uni, book, C, rho=1.0)
    assert np.all(host["status"] == 0)
    dB_ref = np.zeros_like(dB)
    for a in range(book.m):
        P = account(uni, book, a)
        orc = oracle.solve_account(P)
        g_mu, g_B = gradients(P, orc["w"], orc["lam_band"], orc["lam_cap"], C[a])
        # natural scale of a gradient entry: |c| / (gamma d) for one free
        # coordinate (an all-zero reference is an LP-like vertex)
        scale = max(np.abs(g_mu).max(),
                    np.abs(C[a]).max() / (gamma * uni.d.max()))
        assert np.max(np.abs(dmu[a] - g_mu)) <= 1e-6 * scale, a
        assert abs(dmu[a].sum()) <= 1e-9 * scale * uni.n
        dB_ref += g_B
    assert np.max(np.abs(dB - dB_ref)) <= 1e-6 * max(np.abs(dB_ref).max(), 1e-12)


def test_autograd_function():
    import torch
    from paper_2606_23367_amd.solver import Solver, to_device, solve_differentiable
    uni, book = make_config("c4", 1, N=600, M=3, k=8)
    P = to_device(uni, book)
    s = Solver(0)
    mu = P.mu.clone().requires_grad_(True)
    B = P.B.clone().requires_grad_(True)
    w = solve_differentiable(mu, B, P, s, rho=1.0)
    c = torch.randn_like(w)
    (w * c).sum().backward()
    C = c.cpu().numpy()
    for a in range(book.m):
        Pa = account(uni, book, a)
        orc = oracle.solve_account(Pa)
        g_mu, _ = gradients(Pa, orc["w"], orc["lam_band"], orc["lam_cap"], C[a])
        assert np.max(np.abs(mu.grad[a].cpu().numpy() - g_mu)) <= \
            1e-6 * max(np.abs(g_mu).max(), 1e-300)
    assert B.grad is not None and torch.isfinite(B.grad).all()


@pytest.mark.parametrize("gamma", [1000.0, 1.0])
def test_adjoint_at_full_size(gamma):
    """The differentiation workload at its full size (128 accounts over
    N = 5,000 names, k = 60, 10 sector bands): the loss weights only three
    sampled accounts, so dL/dB is the sum of their three reference
    gradients, and dL/dmu of every other account is zero."""
    uni, book = make_config("c4", 0, gamma=gamma)
    sample = (0, 63, 127)
    rng = np.random.default_rng(1)
    C = np.zeros((book.m, uni.n))
    for a in sample:
        C[a] = rng.normal(size=uni.n)
    print(f"case adjoint full size gamma={gamma}", flush=True)
    host, dmu, dB = _gpu_adjoint(uni, book, C, rho=1.0)
    assert np.all(host["status"] == 0)
    others = [a for a in range(book.m) if a not in sample]
    assert np.all(dmu[others] == 0.0)
    dB_ref = np.zeros_like(dB)
    for a in sample:
        P = account(uni, book, a)
        orc = oracle.solve_account(P)
        g_mu, g_B = gradients(P, orc["w"], orc["lam_band"], orc["lam_cap"], C[a])
        scale = max(np.abs(g_mu).max(), np.abs(C[a]).max() / (gamma * uni.d.max()))
        err = float(np.max(np.abs(dmu[a] - g_mu)))
        print("account", a, "free", int(np.count_nonzero(g_mu)), "dmu err", err / scale, flush=True)
        assert err <= 1e-6 * scale, a
        assert abs(dmu[a].sum()) <= 1e-9 * scale * uni.n
        dB_ref += g_B
    assert np.max(np.abs(dB - dB_ref)) <= 1e-6 * max(np.abs(dB_ref).max(), 1e-12)
