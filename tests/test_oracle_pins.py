"""Pins of the float64 oracle against constructions that do not use it.

Every case cites the passage of the paper it checks: the problem class
(Sec. "Benchmark Problem Class", Eq. 1), the external diagnostics (Sec.
"External Diagnostics") and the special objective of the real-data scenarios
(Sec. "Operationally Constrained Real-Data Scenarios").
"""
import numpy as np
import pytest

import oracle
from oracle.problem import account, objective
from oracle.kkt import residuals
from oracle.ipm import solve_ipm
from workloads import make_config
from workloads.books import to_f32_exact

from _pins import (brute_force, closed_form_budget_only, dense_sigma,
                   phi_value, separable_exact)


def _tiny(N, k=3, seed=0, ub=0.23, gamma=1.0, **over):
    uni, book = make_config("c1", seed, N=N, k=k, ub=ub, gamma=gamma, **over)
    return uni, book


# --------------------------------------------------------------------------
# closed form: Eq. 1 with only the budget row
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [8, 60, 300])
@pytest.mark.parametrize("gamma", [1.0, 100.0, 1e4])
def test_closed_form_budget_only(N, gamma):
    uni, book = make_config("c1", 3, N=N, k=5, gamma=gamma)
    w_cf, nu_cf = closed_form_budget_only(uni.B, uni.f, uni.d, book.mu[0],
                                          gamma)
    wide = 4.0 * float(np.max(np.abs(w_cf))) + 1.0   # box inactive
    book.lb[:] = -wide
    book.ub[:] = wide
    P = account(uni, book, 0)
    out = oracle.solve_account(P)
    scale = max(1.0, np.max(np.abs(w_cf)))
    assert np.max(np.abs(out["w"] - w_cf)) <= 1e-10 * scale
    assert abs(out["nu"] - nu_cf) <= 1e-9 * max(1.0, abs(nu_cf))


# --------------------------------------------------------------------------
# brute-force active-set enumeration, N <= 8
# --------------------------------------------------------------------------
def _compare_bf(uni, book, **bf_kw):
    P = account(uni, book, 0)
    out = oracle.solve_account(P)
    w_bf, nu_bf, lam_bf, lamc_bf, nacc = brute_force(
        uni.B, uni.f, uni.d, book.mu[0], float(book.gamma[0]),
        float(book.lb[0]), float(book.ub[0]), **bf_kw)
    assert nacc >= 1
    assert np.max(np.abs(out["w"] - w_bf)) <= 1e-10
    assert abs(objective(P, out["w"]) - objective(P, w_bf)) <= 1e-12
    return out, w_bf


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("gamma", [1.0, 30.0])
def test_brute_force_box(seed, gamma):
    uni, book = _tiny(8, seed=seed, gamma=gamma)
    _compare_bf(uni, book)


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_l1(seed):
    uni, book = _tiny(6, seed=seed, gamma=20.0, kappa=4e-3, w0="dirichlet")
    _compare_bf(uni, book, w0=book.w0[0], kappa=float(book.kappa[0]))


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_tax(seed):
    uni, book = _tiny(4, seed=seed, ub=0.41, gamma=10.0, kappa=1e-3,
                      w0="dirichlet", tax=True)
    ta, tb, ts = book.tax_of(0)
    tax = {int(i): (tb[j], ts[j]) for j, i in enumerate(ta)}
    out, _ = _compare_bf(uni, book, w0=book.w0[0], kappa=float(book.kappa[0]),
                         tax=tax)


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_bands(seed):
    uni, book = _tiny(5, seed=seed, ub=0.37, gamma=5.0, kappa=1e-3,
                      w0="dirichlet", groups=2, band_halfwidth=0.07)
    _compare_bf(uni, book, w0=book.w0[0], kappa=float(book.kappa[0]),
                group=uni.group, band_lo=book.band_lo[0],
                band_hi=book.band_hi[0])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_cap(seed):
    uni, book = _tiny(6, seed=seed, ub=0.31, gamma=3.0, w0="dirichlet")
    tau = float(to_f32_exact(0.35))
    book.tau[:] = tau
    out, w_bf = _compare_bf(uni, book, w0=book.w0[0], tau=tau)
    # the cap binds in these instances (otherwise the pin is vacuous)
    assert abs(np.abs(w_bf - book.w0[0]).sum() - tau) < 1e-12


# --------------------------------------------------------------------------
# separable case B = 0 at the headline width
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name,over", [
    ("c3", dict(N=10000, M=1, k=2)),
    ("c2", dict(N=2000, M=1, k=2, groups=0)),
])
def test_separable_exact(name, over):
    uni, book = make_config(name, 7, **over)
    uni.B[:] = 0.0
    P = account(uni, book, 0)
    out = oracle.solve_account(P)
    ta, tb, ts = book.tax_of(0)
    tax = {int(i): (tb[j], ts[j]) for j, i in enumerate(ta)}
    w_ex, nu_ex, lam_ex = separable_exact(
        uni.d, book.mu[0], float(book.gamma[0]), float(book.lb[0]),
        float(book.ub[0]), book.eligible[0], book.w0[0],
        float(book.kappa[0]), tax, float(book.tau[0]))
    assert np.max(np.abs(out["w"] - w_ex)) <= 1e-11
    if np.isfinite(book.tau[0]):
        assert lam_ex > 0                       # cap binding: not vacuous
        assert abs(out["lam_cap"] - lam_ex) <= 1e-8 * max(lam_ex, 1e-6)


# --------------------------------------------------------------------------
# the two linear-algebra routes of the interior-point method agree
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name,over", [
    ("c2", dict(N=300, M=1, k=8)),
    ("c3", dict(N=500, M=1, k=10)),
    ("c4", dict(N=300, M=1, k=6)),
])
def test_routes_agree(name, over):
    uni, book = make_config(name, 1, **over)
    P = account(uni, book, 0)
    r1 = solve_ipm(P, route="schur")
    r2 = solve_ipm(P, route="sparse")
    assert r1.converged and r2.converged
    assert np.max(np.abs(r1.w - r2.w)) <= 1e-10


# --------------------------------------------------------------------------
# external diagnostics (Sec. "External Diagnostics")
# --------------------------------------------------------------------------
def test_residuals_zero_at_closed_form_and_detect_mistakes():
    uni, book = make_config("c1", 5, N=40, k=4)
    w, nu = closed_form_budget_only(uni.B, uni.f, uni.d, book.mu[0], 1.0)
    book.lb[:] = -100.0
    book.ub[:] = 100.0
    P = account(uni, book, 0)
    r = residuals(P, w, nu)
    assert r["r_prim"] < 1e-13 and r["r_dual"] < 1e-10 and r["r_comp"] == 0
    # a wrong budget multiplier shows in stationarity
    assert residuals(P, w, nu + 1e-4)["r_dual"] > 1e-4
    # a moved weight shows in the budget residual and stationarity
    w2 = w.copy()
    w2[3] += 1e-5
    r2 = residuals(P, w2, nu)
    assert abs(r2["r_budget"] - 1e-5) < 1e-12 and r2["r_dual"] > 1e-9


def test_residuals_cap_and_band_signs():
    uni, book = make_config("c3", 2, N=400, M=1, k=6)
    P = account(uni, book, 0)
    out = oracle.solve_account(P)
    assert out["lam_cap"] > 0
    ok = residuals(P, out["w"], out["nu"], out["lam_band"], out["lam_cap"])
    assert max(ok["r_prim"], ok["r_dual"], ok["r_comp"]) < 1e-10
    bad = residuals(P, out["w"], out["nu"], out["lam_band"], -out["lam_cap"])
    assert bad["r_dual"] > 1e-3
    uni, book = make_config("c2", 2, N=300, M=1, k=6)
    P = account(uni, book, 0)
    out = oracle.solve_account(P)
    g = int(np.argmax(np.abs(out["lam_band"])))
    assert abs(out["lam_band"][g]) > 1e-6        # some band binds
    flipped = out["lam_band"].copy()
    flipped[g] = -flipped[g]
    assert residuals(P, out["w"], out["nu"], flipped)["r_dual"] > 1e-4


def test_objective_matches_dense_evaluation():
    uni, book = make_config("c3", 4, N=300, M=1, k=5)
    P = account(uni, book, 0)
    rng = np.random.default_rng(0)
    w = rng.uniform(0, 0.01, size=300)
    S = dense_sigma(uni.B, uni.f, uni.d)
    ta, tb, ts = book.tax_of(0)
    tax = {int(i): (tb[j], ts[j]) for j, i in enumerate(ta)}
    ref = 0.5 * w @ S @ w - book.mu[0] @ w
    for i in range(300):
        t = tax.get(i, (None, None))
        ref += phi_value(w[i], book.w0[0, i], float(book.kappa[0]), *t)
    assert abs(objective(P, w) - ref) < 1e-15


def test_e7_objective_is_the_gamma2_instance():
    """The real-data scenario's objective ||B^T w||^2 + w^T diag(d) w
    - mu^T w + g ||w - w0||_1 is this build's f with gamma = 2, F = I and
    kappa = g (Sec. "Operationally Constrained Real-Data Scenarios")."""
    uni, book = make_config("c2", 0, N=200, M=1, k=20, groups=0,
                            gamma=2.0, kappa=0.005)
    uni.f[:] = 1.0
    P = account(uni, book, 0)
    rng = np.random.default_rng(1)
    for _ in range(5):
        w = rng.dirichlet(np.ones(200))
        g = float(book.kappa[0])
        e7 = np.sum((uni.B.T @ w) ** 2) + w @ (uni.d * w) - book.mu[0] @ w \
            + g * np.abs(w - book.w0[0]).sum()
        assert abs(objective(P, w) - e7) < 1e-15


# --------------------------------------------------------------------------
# every configuration shape (scaled down) is certified by the oracle
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name,over", [
    ("c1", {}),
    ("c2", dict(N=400, M=3, k=10)),
    ("c3", dict(N=800, M=3, k=12)),
    ("c4", dict(N=500, M=2, k=8)),
    ("c4", dict(N=500, M=2, k=8, gamma=1.0)),
    ("c5", dict(N=3000, M=1, k=10, held=(150, 150))),
])
@pytest.mark.parametrize("seed", [0, 1])
def test_oracle_certifies_configs(name, over, seed):
    uni, book = make_config(name, seed, **over)
    for a in range(book.m):
        P = account(uni, book, a)
        out = oracle.solve_account(P)
        r = out["res"]
        assert out["method"] == "crossover"
        assert r["r_prim"] < 1e-11 and r["r_dual"] < 1e-11 \
            and r["r_comp"] < 1e-11
        # the paper's quality gates (Sec. "Quality Gates and Failure
        # Vocabulary"): budget <= 1e-4, bound violation <= 1e-6
        assert r["r_budget"] <= 1e-4 and r["r_box"] <= 1e-6


def test_crossover_recovers_multipliers_at_degenerate_vertex():
    """At an LP-like vertex the free rows do not pin every multiplier; the
    crossover must still return multipliers inside every fixed coordinate's
    subdifferential even from perturbed interior-point estimates."""
    from oracle.crossover import crossover
    for name, over in [("c1", {}), ("c3", dict(N=600, M=1, k=8))]:
        for seed in (0, 1, 2):
            uni, book = make_config(name, seed, **over)
            P = account(uni, book, 0)
            r = solve_ipm(P)
            for d_nu, d_lam in [(2e-4, 0.0), (-3e-4, 1e-3), (1e-5, -1e-3)]:
                out = crossover(P, r.w, r.nu + d_nu, r.lam_band,
                                max(r.lam_cap + d_lam, 0.0))
                res = out["res"]
                assert out["method"] == "crossover"
                assert max(res["r_prim"], res["r_dual"], res["r_comp"]) < 1e-11
