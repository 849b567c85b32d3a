"""One account's instance of Eq. 1 as plain float64 arrays (oracle side).

The build's instantiation of the paper's problem class (Sec. "Benchmark
Problem Class", Eq. 1) is

    min_w  (gamma/2) w^T Sigma w - mu^T w + sum_i phi_i(w_i - w0_i)
    s.t.   1^T w = 1,  lb <= w_i <= ub (w_i = 0 if excluded),
           band_lo <= A w <= band_hi  (A one-hot by group label),
           sum_i |w_i - w0_i| <= tau,

with Sigma = B diag(f) B^T + diag(d) and the separable trade cost
phi_i(D) = kappa |D| + T_i((-D)_+), T_i the convex piecewise-linear tax on the
sale amount.  This is Eq. 1 with Q = gamma Sigma, eta = 1, benchmark weights
w_b = 0, no extra regulariser R and no policy halfspaces (D_a = I).

Test infrastructure only: nothing in the product path may import this package.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class AccountProblem:
    B: np.ndarray
    f: np.ndarray
    d: np.ndarray
    group: Optional[np.ndarray]
    n_groups: int
    mu: np.ndarray
    w0: np.ndarray
    lb: float
    ub: float
    eligible: np.ndarray
    gamma: float
    kappa: float
    tau: float
    band_lo: Optional[np.ndarray]
    band_hi: Optional[np.ndarray]
    tax_asset: np.ndarray
    tax_brk: np.ndarray
    tax_slope: np.ndarray

    @property
    def n(self):
        return self.B.shape[0]

    @property
    def k(self):
        return self.B.shape[1]


def account(uni, book, a: int) -> AccountProblem:
    """Extract account ``a`` of a (Universe, Book) pair."""
    ta, tb, ts = book.tax_of(a)
    G = uni.n_groups if book.band_lo is not None else 0
    return AccountProblem(
        B=uni.B, f=uni.f, d=uni.d,
        group=uni.group if G else None, n_groups=G,
        mu=book.mu[a], w0=book.w0[a],
        lb=float(book.lb[a]), ub=float(book.ub[a]),
        eligible=book.eligible[a],
        gamma=float(book.gamma[a]), kappa=float(book.kappa[a]),
        tau=float(book.tau[a]),
        band_lo=None if not G else book.band_lo[a],
        band_hi=None if not G else book.band_hi[a],
        tax_asset=np.asarray(ta, dtype=np.int64),
        tax_brk=np.asarray(tb, dtype=np.float64).reshape(-1, 3),
        tax_slope=np.asarray(ts, dtype=np.float64).reshape(-1, 4),
    )


def sigma_times(P: AccountProblem, w):
    """Sigma w = B (f * (B^T w)) + d * w, in float64 (factor structure of the
    risk operator, Sec. "Benchmark Problem Class")."""
    return P.B @ (P.f * (P.B.T @ w)) + P.d * w


def tax_cost(brk, slope, s):
    """T(s) for sale amount s >= 0: convex piecewise-linear, slope[j] on the
    j-th lot, the last slope continuing past the last breakpoint."""
    s = max(float(s), 0.0)
    edges = [0.0, brk[0], brk[1], brk[2], np.inf]
    total = 0.0
    for j in range(4):
        lo, hi = edges[j], edges[j + 1]
        if s > lo:
            total += slope[j] * (min(s, hi) - lo)
    return total


def trade_cost(P: AccountProblem, w):
    """sum_i phi_i(w_i - w0_i): L1 turnover plus sale-side tax."""
    dw = w - P.w0
    total = P.kappa * np.abs(dw).sum()
    for idx, i in enumerate(P.tax_asset):
        total += tax_cost(P.tax_brk[idx], P.tax_slope[idx], -dw[i])
    return total


def objective(P: AccountProblem, w):
    """f(w) of the build's Eq. 1 instance, recomputed in float64."""
    w = np.asarray(w, dtype=np.float64)
    return 0.5 * P.gamma * float(w @ sigma_times(P, w)) - float(P.mu @ w) \
        + trade_cost(P, w)


def objective_scale(P: AccountProblem, w):
    """Denominator for relative objective errors: |f| or the sum of the
    magnitudes of its terms, whichever is larger (never zero)."""
    w = np.asarray(w, dtype=np.float64)
    risk = 0.5 * P.gamma * float(w @ sigma_times(P, w))
    ret = abs(float(P.mu @ w))
    tc = trade_cost(P, w)
    return max(abs(risk - float(P.mu @ w) + tc), risk + ret + tc, 1e-300)


def kinks_and_slopes(P: AccountProblem, i: int, lam_cap: float = 0.0):
    """Kink points (ascending, in weight space) and the slopes of
    phi_i + lam_cap |. - w0_i| on each piece (one more slope than kinks).

    Held, taxed assets: kinks at w0 - b3 < w0 - b2 < w0 - b1 < w0; slopes
    -(kappa+lam+s3), ..., -(kappa+lam+s0) on the sale side and kappa+lam on
    the buy side.  Other assets: one kink at w0 with slopes -/+(kappa+lam).
    """
    w0 = float(P.w0[i])
    kl = P.kappa + lam_cap
    hit = np.nonzero(P.tax_asset == i)[0]
    if len(hit):
        j = int(hit[0])
        b = P.tax_brk[j]
        s = P.tax_slope[j]
        kinks = np.array([w0 - b[2], w0 - b[1], w0 - b[0], w0])
        slopes = np.array([-(kl + s[3]), -(kl + s[2]), -(kl + s[1]),
                           -(kl + s[0]), kl])
    else:
        kinks = np.array([w0])
        slopes = np.array([-kl, kl])
    return kinks, slopes
