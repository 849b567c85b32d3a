"""Pins of the float64 reference gradient (implicit differentiation of the
KKT system at the optimum of the build's Eq. 1 instance) against central
finite differences of the oracle and against exact invariants."""
import numpy as np
import pytest

import oracle
from oracle.adjoint import gradients
from oracle.problem import account
from workloads import make_config


def _solve(uni, book, a=0):
    P = account(uni, book, a)
    out = oracle.solve_account(P)
    # an exact point: the crossover's, or an interior-point iterate that
    # already certifies at round-off level
    r = out["res"]
    assert max(r["r_prim"], r["r_dual"], r["r_comp"]) <= 1e-13, (out["method"], r)
    return P, out


@pytest.mark.parametrize("name,over", [
    ("c4", dict(N=120, M=1, k=6)),                 # gamma = 1000, bands, L1
    ("c4", dict(N=120, M=1, k=6, gamma=1.0)),
    ("c3", dict(N=300, M=1, k=6)),                 # tax + cap
    # the rest of Eq. 1: halfspace rows, per-asset bounds, benchmark, eta
    ("c4", dict(N=120, M=1, k=6, halfspaces=3, asset_bounds=True, benchmark=True)),
])
def test_dmu_matches_central_differences(name, over):
    uni, book = make_config(name, 11, **over)
    P, out = _solve(uni, book)
    rng = np.random.default_rng(3)
    c = rng.normal(size=uni.n)
    dmu, _ = gradients(P, out["w"], out["lam_band"], out["lam_cap"], c)
    h = 1e-7
    idx = list(np.nonzero(dmu)[0][:6]) + list(rng.choice(uni.n, 4, replace=False))
    checked = 0
    for i in idx:
        vals = []
        pats = []
        for s in (+1, -1):
            b2 = make_config(name, 11, **over)[1]
            b2.mu[0, i] += s * h
            o2 = oracle.solve_account(account(uni, b2, 0))
            vals.append(c @ o2["w"])
            pats.append(np.round(o2["w"], 9) == np.round(out["w"], 9))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - dmu[i]) <= 1e-5 * max(1.0, abs(dmu[i])), (i, fd, dmu[i])
        checked += 1
    assert checked == len(idx) and np.count_nonzero(dmu) >= 1


@pytest.mark.parametrize("over", [dict(), dict(halfspaces=2, benchmark=True)])
def test_dB_matches_central_differences(over):
    """(With halfspace rows, they are data of their own: perturbing B does
    not move them.)"""
    uni, book = make_config("c4", 12, N=100, M=1, k=5, **over)
    P, out = _solve(uni, book)
    rng = np.random.default_rng(4)
    c = rng.normal(size=uni.n)
    _, dB = gradients(P, out["w"], out["lam_band"], out["lam_cap"], c)
    h = 1e-7
    support = np.nonzero(out["w"])[0]
    for i in list(support[:4]) + [int(rng.integers(uni.n))]:
        for j in (0, 3):
            vals = []
            for s in (+1, -1):
                u2 = make_config("c4", 12, N=100, M=1, k=5, **over)[0]
                u2.B[i, j] += s * h
                o2 = oracle.solve_account(account(u2, book, 0))
                vals.append(c @ o2["w"])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - dB[i, j]) <= 1e-5 * max(1.0, abs(dB[i, j])), \
                (i, j, fd, dB[i, j])


def test_gradient_invariants():
    uni, book = make_config("c4", 13, N=200, M=1, k=6)
    P, out = _solve(uni, book)
    rng = np.random.default_rng(5)
    c1, c2 = rng.normal(size=(2, uni.n))
    g1, _ = gradients(P, out["w"], out["lam_band"], out["lam_cap"], c1)
    g2, _ = gradients(P, out["w"], out["lam_band"], out["lam_cap"], c2)
    # shifting mu by s*1 is absorbed by the budget multiplier
    assert abs(g1.sum()) <= 1e-9 * np.abs(g1).sum()
    # dw/dmu is symmetric:  c2^T J c1 = c1^T J c2
    assert abs(c2 @ g1 - c1 @ g2) <= 1e-9 * (abs(c2 @ g1) + 1e-300)
