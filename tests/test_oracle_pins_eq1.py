"""Pins of the float64 oracle on the rest of Eq. 1 (Sec. "Benchmark Problem
Class"): policy halfspaces G w <= h (rows shared by the book, bounds per
account, either side possibly infinite), per-asset bounds lb_i <= w_i <= ub_i
and the benchmark-relative risk (1/2)(w - w_b)^T Q (w - w_b) with the return
scale eta.  Each case compares the oracle with a construction that does not
use it: the closed form of the budget-only problem, brute-force active-set
enumeration (tests/_pins.py), a dense evaluation of the objective, or the
other linear-algebra route.
"""
import numpy as np
import pytest

import oracle
from oracle.problem import account, objective
from oracle.kkt import residuals
from workloads import make_config
from workloads.books import to_f32_exact

from _pins import brute_force, closed_form_benchmark, dense_sigma, phi_value


def _bf_args(uni, book, a=0, **extra):
    """brute_force arguments of account a, straight from the book arrays."""
    kw = dict(w0=book.w0[a], kappa=float(book.kappa[a]), tau=float(book.tau[a]))
    if book.band_lo is not None:
        kw.update(group=uni.group, band_lo=book.band_lo[a], band_hi=book.band_hi[a])
    if book.half_lo is not None:
        kw.update(half=uni.half, half_lo=book.half_lo[a], half_hi=book.half_hi[a])
    if book.wb is not None:
        kw.update(wb=book.wb[a], eta=float(book.eta[a]))
    ta, tb, ts = book.tax_of(a)
    if len(ta):
        kw["tax"] = {int(i): (tb[j], ts[j]) for j, i in enumerate(ta)}
    lb = book.lb_asset[a] if book.lb_asset is not None else float(book.lb[a])
    ub = book.ub_asset[a] if book.ub_asset is not None else float(book.ub[a])
    if book.lb_asset is not None:
        lb = np.where(book.eligible[a], lb, 0.0)
        ub = np.where(book.eligible[a], ub, 0.0)
    kw.update(extra)
    return (uni.B, uni.f, uni.d, book.mu[a], float(book.gamma[a]), lb, ub), kw


def _compare_bf(uni, book, a=0):
    P = account(uni, book, a)
    out = oracle.solve_account(P)
    args, kw = _bf_args(uni, book, a)
    w_bf, nu_bf, lam_bf, lamc_bf, nacc = brute_force(*args, **kw)
    assert nacc >= 1
    assert np.max(np.abs(out["w"] - w_bf)) <= 1e-10, np.max(np.abs(out["w"] - w_bf))
    assert abs(objective(P, out["w"]) - objective(P, w_bf)) <= 1e-12
    r = out["res"]
    assert max(r["r_prim"], r["r_dual"], r["r_comp"]) <= 1e-10
    return P, out, w_bf, lam_bf


# --------------------------------------------------------------------------
# benchmark-relative risk, budget only: closed form
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [8, 60, 300])
@pytest.mark.parametrize("gamma", [1.0, 100.0])
def test_closed_form_with_benchmark(N, gamma):
    uni, book = make_config("c1", 4, N=N, k=5, gamma=gamma, benchmark=True)
    wb, eta = book.wb[0], float(book.eta[0])
    assert np.abs(wb).sum() > 0.5 and eta != 1.0
    w_cf, nu_cf = closed_form_benchmark(uni.B, uni.f, uni.d, book.mu[0], gamma, wb, eta)
    wide = 4.0 * float(np.max(np.abs(w_cf))) + 1.0   # box inactive
    book.lb[:] = -wide
    book.ub[:] = wide
    P = account(uni, book, 0)
    out = oracle.solve_account(P)
    scale = max(1.0, np.max(np.abs(w_cf)))
    assert np.max(np.abs(out["w"] - w_cf)) <= 1e-10 * scale
    assert abs(out["nu"] - nu_cf) <= 1e-9 * max(1.0, abs(nu_cf))


# --------------------------------------------------------------------------
# brute force, N <= 6
# --------------------------------------------------------------------------
def _tiny(N, seed, **over):
    return make_config("c1", seed, N=N, k=3, **over)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_brute_force_halfspaces(seed):
    """Two factor-exposure rows (the second one-sided), L1 trade cost."""
    uni, book = _tiny(5, seed, ub=0.37, gamma=5.0, kappa=1e-3, w0="dirichlet",
                      halfspaces=2, half_halfwidth=4e-3)
    assert np.isinf(book.half_lo[0, 1]) and np.isfinite(book.half_hi[0, 1])
    _compare_bf(uni, book)


def test_some_halfspace_binds():
    """The halfspace pins above are not vacuous: a row binds in some seed."""
    binds = 0
    for seed in range(4):
        uni, book = _tiny(5, seed, ub=0.37, gamma=5.0, kappa=1e-3, w0="dirichlet",
                          halfspaces=2, half_halfwidth=4e-3)
        args, kw = _bf_args(uni, book)
        w_bf, _, lam, _, _ = brute_force(*args, **kw)
        Hw = uni.half @ w_bf
        bind = np.minimum(np.abs(Hw - book.half_lo[0]), np.abs(Hw - book.half_hi[0]))
        binds += int(np.min(bind) < 1e-12 and np.max(np.abs(lam)) > 0.0)
    assert binds >= 2


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_asset_bounds(seed):
    """Per-asset upper bounds and one forced minimum holding."""
    uni, book = _tiny(6, seed, ub=0.41, gamma=8.0, kappa=2e-3, w0="dirichlet",
                      asset_bounds=True)
    book.lb_asset[0, 2] = float(to_f32_exact(0.3 * book.ub_asset[0, 2]))
    P, out, w_bf, _ = _compare_bf(uni, book)
    # some per-asset bound is active (the pin is not vacuous)
    at = np.isclose(w_bf, book.ub_asset[0], atol=1e-12) | np.isclose(w_bf, book.lb_asset[0],
                                                                    atol=1e-12)
    assert at[book.lb_asset[0] > 0].any() or (at & (book.ub_asset[0] < 0.41)).any()


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_benchmark(seed):
    uni, book = _tiny(6, seed, ub=0.33, gamma=40.0, kappa=3e-3, w0="dirichlet",
                      benchmark=True)
    _compare_bf(uni, book)


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_everything(seed):
    """Halfspaces, per-asset bounds, benchmark, L1, a binding turnover cap."""
    uni, book = _tiny(5, seed, ub=0.45, gamma=10.0, kappa=1e-3, w0="dirichlet",
                      halfspaces=2, half_halfwidth=6e-3, asset_bounds=True, benchmark=True)
    tau = float(to_f32_exact(0.3))
    book.tau[:] = tau
    P, out, w_bf, _ = _compare_bf(uni, book)
    assert abs(np.abs(w_bf - book.w0[0]).sum() - tau) < 1e-12     # the cap binds


# --------------------------------------------------------------------------
# objective and checker
# --------------------------------------------------------------------------
def test_objective_with_benchmark_matches_dense_evaluation():
    uni, book = make_config("c2", 2, N=40, M=1, k=4, benchmark=True, halfspaces=2)
    P = account(uni, book, 0)
    rng = np.random.default_rng(5)
    w = rng.dirichlet(np.ones(uni.n))
    Q = float(book.gamma[0]) * dense_sigma(uni.B, uni.f, uni.d)
    e = w - book.wb[0]
    dense = 0.5 * e @ Q @ e - float(book.eta[0]) * book.mu[0] @ w + \
        sum(phi_value(w[i], book.w0[0, i], float(book.kappa[0])) for i in range(uni.n))
    assert abs(objective(P, w) - dense) <= 1e-14 * max(1.0, abs(dense))


def test_residuals_detect_halfspace_mistakes():
    """At the oracle's optimum the checker is ~0; it flags a weight moved
    across a binding halfspace, and a halfspace multiplier of the wrong
    sign."""
    found = None
    for seed in range(6):
        uni, book = make_config("c2", seed, N=120, M=1, k=6, groups=0, halfspaces=3,
                                half_halfwidth=2e-3)
        P = account(uni, book, 0)
        out = oracle.solve_account(P)
        lam = out["lam_band"]
        if np.max(np.abs(lam)) > 1e-8:
            found = (uni, book, P, out)
            break
    assert found is not None, "no binding halfspace in the seeds tried"
    uni, book, P, out = found
    r0 = residuals(P, out["w"], out["nu"], out["lam_band"], out["lam_cap"])
    assert max(r0["r_prim"], r0["r_dual"], r0["r_comp"]) <= 1e-10
    j = int(np.argmax(np.abs(out["lam_band"])))
    # move weight along the row's steepest direction (budget kept)
    hrow = uni.half[j]
    i_up, i_dn = int(np.argmax(hrow)), int(np.argmin(hrow))
    w2 = out["w"].copy()
    step = 1e-4 * np.sign(out["lam_band"][j])
    w2[i_up] += step
    w2[i_dn] -= step
    assert residuals(P, w2, out["nu"], out["lam_band"], out["lam_cap"])["r_exposure"] > 1e-6
    lam_bad = out["lam_band"].copy()
    lam_bad[j] = -lam_bad[j]
    r_bad = residuals(P, out["w"], out["nu"], lam_bad, out["lam_cap"])
    assert max(r_bad["r_dual"], r_bad["r_comp"]) > 1e-6


@pytest.mark.parametrize("seed", [0, 1])
def test_routes_agree_full_eq1(seed):
    uni, book = make_config("c2", seed, N=300, M=1, k=8, halfspaces=3, asset_bounds=True,
                            benchmark=True)
    P = account(uni, book, 0)
    a = oracle.solve_account(P, route="schur")
    b = oracle.solve_account(P, route="sparse")
    assert np.max(np.abs(a["w"] - b["w"])) <= 1e-10
    for out in (a, b):
        r = out["res"]
        assert max(r["r_prim"], r["r_dual"], r["r_comp"]) <= 1e-11


@pytest.mark.parametrize("name,over", [
    ("c3", dict(N=1500, M=1, k=12, halfspaces=4, asset_bounds=True, benchmark=True)),
    ("c2", dict(N=800, M=1, k=10, halfspaces=5, benchmark=True)),
])
def test_oracle_certifies_full_eq1(name, over):
    uni, book = make_config(name, 3, **over)
    P = account(uni, book, 0)
    out = oracle.solve_account(P)
    r = out["res"]
    assert max(r["r_prim"], r["r_dual"], r["r_comp"]) <= 1e-11, r
