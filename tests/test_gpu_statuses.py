"""Statuses the paper's failure vocabulary names for returns that are not
certified (Sec. "Quality Gates and Failure Vocabulary"; status table of
Sec. "Status Vocabulary and Objective Agreement"), forced from the host:
an iteration cap, a time limit and a failed device allocation.  Plus the
state a warm start carries across handles, the graph a repeated call
replays, and the autograd guard against a replaced solve."""
import ctypes

import numpy as np
import pytest

from oracle.problem import account
from oracle.kkt import residuals
from workloads import make_config
from _gpu_helpers import run_gpu, check_account, check_reported_diagnostics

pytestmark = pytest.mark.gpu

SOLVED, FEASIBLE_UNCERTIFIED, MAX_ITER, TIME_LIMIT = 0, 1, 2, 3


def _gates(r):
    """The paper's quality gates: budget residual <= 1e-4 and bound
    violations (box, exposure bands, turnover cap) <= 1e-6."""
    return r["r_budget"] <= 1e-4 and max(r["r_box"], r["r_exposure"], r["r_turnover"]) <= 1e-6


def _check_returned(uni, book, host, a):
    P = account(uni, book, a)
    lam_band = host["lam_band"][a] if P.n_groups else None
    r = residuals(P, host["w"][a], host["nu"][a], lam_band, host["lam_cap"][a])
    check_reported_diagnostics(host, a, r)
    return r


@pytest.mark.parametrize("max_iter", [1, 20])
def test_iteration_cap(max_iter):
    """Stopped after max_iter iterations: every account is certified, or
    returns its best iterate as FEASIBLE_UNCERTIFIED when the gates pass
    and MAX_ITER when they fail -- as the CPU checker sees them."""
    uni, book = make_config("c3", 21, N=1300, M=9, k=16)
    print(f"case max_iter={max_iter}", flush=True)
    host, st = run_gpu(uni, book, rho=5.0, max_iter=max_iter, check_every=50)
    assert st["iterations"] == max_iter
    assert np.all(host["iters"] <= max_iter)
    stat = host["status"]
    assert set(stat.tolist()) <= {SOLVED, FEASIBLE_UNCERTIFIED, MAX_ITER}, stat
    assert np.any(stat != SOLVED), stat
    for a in range(book.m):
        r = _check_returned(uni, book, host, a)
        if stat[a] == SOLVED:
            check_account(uni, book, a, host)
        elif stat[a] == FEASIBLE_UNCERTIFIED:
            assert _gates(r), (a, r)
            assert max(r["r_prim"], r["r_dual"], r["r_comp"]) > 1e-6, (a, r)
        else:
            assert not _gates(r), (a, r)


def test_time_limit():
    """A time limit shorter than one block: the call stops after the first
    certification pass; accounts that pass then are certified, the others
    return their best iterate as TIME_LIMIT (gates fail) or
    FEASIBLE_UNCERTIFIED (gates pass)."""
    uni, book = make_config("c3", 22, N=1300, M=9, k=16)
    print("case time limit", flush=True)
    host, st = run_gpu(uni, book, rho=5.0, check_every=10, time_limit_ms=1e-3)
    assert st["iterations"] == 10
    stat = host["status"]
    assert set(stat.tolist()) <= {SOLVED, FEASIBLE_UNCERTIFIED, TIME_LIMIT}, stat
    assert np.any(stat != SOLVED), stat
    for a in range(book.m):
        r = _check_returned(uni, book, host, a)
        if stat[a] == TIME_LIMIT:
            assert not _gates(r), (a, r)
        elif stat[a] == FEASIBLE_UNCERTIFIED:
            assert _gates(r), (a, r)


@pytest.mark.parametrize("where", ["first", "middle", "last"])
def test_allocation_failure_writes_nothing(where):
    """A workspace request of the call fails (the first, one in the middle,
    the last -- the held records, sized after the validation pass ran):
    FQP_ERR_ALLOC, every output left as it was; the handle then solves
    normally."""
    import torch
    from paper_2606_23367_amd import _lib
    from paper_2606_23367_amd.solver import Solver, to_device
    uni, book = make_config("c3", 23, N=900, M=5, k=8)
    P = to_device(uni, book)
    s = Solver(0)
    s.solve(P, rho=5.0)
    torch.cuda.synchronize()
    n_req = s.stats()["workspace_requests"]
    assert n_req > 10
    fail_at = {"first": 1, "middle": n_req // 2, "last": n_req}[where]
    m, n = book.m, uni.n
    out = dict(w=torch.full((m, n), 7.0, dtype=torch.float64, device="cuda:0"),
               status=torch.full((m,), 77, dtype=torch.int32, device="cuda:0"),
               iters=torch.full((m,), 77, dtype=torch.int32, device="cuda:0"))
    for key in ("r_prim", "r_dual", "r_comp", "obj", "nu", "lam_cap"):
        out[key] = torch.full((m,), 7.0, dtype=torch.float64, device="cuda:0")
    out["lam_band"] = torch.full((m, 1), 7.0, dtype=torch.float64, device="cuda:0")
    print(f"case fail_at={fail_at}", flush=True)
    with pytest.raises(RuntimeError, match="device allocation failed"):
        s.solve(P, out=out, rho=5.0, debug_fail_alloc=fail_at)
    torch.cuda.synchronize()
    assert torch.all(out["w"] == 7.0) and torch.all(out["status"] == 77)
    assert torch.all(out["iters"] == 77) and torch.all(out["obj"] == 7.0)
    host = {k: v.cpu().numpy() for k, v in s.solve(P, rho=5.0).items()}
    torch.cuda.synchronize()
    for a in range(m):
        check_account(uni, book, a, host)
    assert _lib.FEASIBLE_UNCERTIFIED == FEASIBLE_UNCERTIFIED


def test_repeated_call_replays_the_kept_graph():
    import torch
    from paper_2606_23367_amd.solver import Solver, to_device
    uni, book = make_config("c3", 24, N=1500, M=12, k=12)
    P = to_device(uni, book)
    s = Solver(0)
    h1 = {k: v.cpu().numpy() for k, v in s.solve(P, rho=5.0).items()}
    assert s.stats()["graph_reused"] == 0
    h2 = {k: v.cpu().numpy() for k, v in s.solve(P, rho=5.0).items()}
    assert s.stats()["graph_reused"] == 1
    torch.cuda.synchronize()
    assert np.array_equal(h1["w"], h2["w"]) and np.array_equal(h1["iters"], h2["iters"])
    # another schedule: a new capture, same optimum
    h3 = {k: v.cpu().numpy() for k, v in s.solve(P, rho=5.0, check_every=40).items()}
    assert s.stats()["graph_reused"] == 0
    for a in (0, 11):
        check_account(uni, book, a, h3)
    ph = s.stats()["phase_ms"]
    assert all(x >= 0.0 for x in ph) and ph[1] > 0.0 and ph[2] > 0.0


def test_warm_state_across_handles():
    """The ADMM state of one handle's solve seeds another handle's solve of
    the next day's book: same optimum (checked against the oracle), fewer
    iterations than cold."""
    import dataclasses
    import torch
    from paper_2606_23367_amd.solver import Solver, to_device
    from workloads.books import to_f32_exact
    uni, book = make_config("c3", 25, N=1300, M=9, k=16)
    rng = np.random.default_rng(26)
    book2 = dataclasses.replace(book, mu=to_f32_exact(book.mu + rng.normal(0.0, 1e-4, book.mu.shape)))
    P1, P2 = to_device(uni, book), to_device(uni, book2)
    sched = dict(rho=5.0, check_every=50)
    s1 = Solver(0)
    state = s1.solve(P1, want_state=True, **sched)["state"].clone()
    s1.close()
    cold = {k: v.cpu().numpy() for k, v in Solver(0).solve(P2, **sched).items()}
    s2 = Solver(0)
    warm = {k: v.cpu().numpy() for k, v in
            s2.solve(P2, warm_state=state, warm_start=1, **sched).items()}
    torch.cuda.synchronize()
    for a in range(book2.m):
        check_account(uni, book2, a, warm)
    print("iterations cold", cold["iters"].tolist(), "warm", warm["iters"].tolist(), flush=True)
    assert int(warm["iters"].sum()) < int(cold["iters"].sum())


def test_backward_after_another_solve_is_refused():
    """The adjoint differentiates the handle's last solve: a backward through
    an earlier forward on the same Solver must fail loudly."""
    import torch
    from paper_2606_23367_amd.solver import Solver, to_device, solve_differentiable
    uni, book = make_config("c4", 27, N=600, M=3, k=8)
    uni2, book2 = make_config("c4", 28, N=600, M=3, k=8)
    P, P2 = to_device(uni, book), to_device(uni2, book2)
    s = Solver(0)
    mu = P.mu.clone().requires_grad_(True)
    B = P.B.clone().requires_grad_(True)
    w1 = solve_differentiable(mu, B, P, s, rho=1.0)
    mu2 = P2.mu.clone().requires_grad_(True)
    B2 = P2.B.clone().requires_grad_(True)
    w2 = solve_differentiable(mu2, B2, P2, s, rho=1.0)
    with pytest.raises(RuntimeError, match="solved another book"):
        (w1.sum() + w2.sum()).backward()
    # one Solver per differentiable call works
    s1, s2 = Solver(0), Solver(0)
    mu.grad = None
    w1 = solve_differentiable(mu, B, P, s1, rho=1.0)
    w2 = solve_differentiable(mu2, B2, P2, s2, rho=1.0)
    (w1.sum() + 2.0 * w2.sum()).backward()
    torch.cuda.synchronize()
    assert torch.isfinite(mu.grad).all() and torch.isfinite(mu2.grad).all()
