"""One account's instance of Eq. 1 as plain float64 arrays (oracle side).

The build's instantiation of the paper's problem class (Sec. "Benchmark
Problem Class", Eq. 1) is

    min_w  (gamma/2)(w - w_b)^T Sigma (w - w_b) - eta mu^T w
           + sum_i phi_i(w_i - w0_i)
    s.t.   1^T w = 1,  lb_i <= w_i <= ub_i (w_i = 0 if excluded),
           band_lo <= A w <= band_hi  (A one-hot by group label),
           half_lo <= H w <= half_hi  (policy halfspace rows),
           sum_i |w_i - w0_i| <= tau,

with Sigma = B diag(f) B^T + diag(d) and the separable trade cost
phi_i(D) = kappa |D| + T_i((-D)_+), T_i the convex piecewise-linear tax on the
sale amount.  This is Eq. 1 with Q = gamma Sigma, no extra regulariser R and
D_a = I; the policy halfspaces G_a w <= h_a are rows H shared by the book
with per-account two-sided bounds (one side may be infinite).  Without
w_b and eta the instance is the budget / box / band / cap / tax problem.

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
    # the rest of Eq. 1: lb / ub may also be (n,) arrays; halfspace rows
    # (H, n) with bounds (H,) (infinite: one-sided); benchmark w_b, eta
    half: Optional[np.ndarray] = None
    half_lo: Optional[np.ndarray] = None
    half_hi: Optional[np.ndarray] = None
    wb: Optional[np.ndarray] = None
    eta: float = 1.0

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
    H = getattr(uni, "n_half", 0) if getattr(book, "half_lo", None) is not None else 0
    lb_a = getattr(book, "lb_asset", None)
    ub_a = getattr(book, "ub_asset", None)
    wb = getattr(book, "wb", None)
    eta = getattr(book, "eta", None)
    return AccountProblem(
        B=uni.B, f=uni.f, d=uni.d,
        group=uni.group if G else None, n_groups=G,
        mu=book.mu[a], w0=book.w0[a],
        lb=float(book.lb[a]) if lb_a is None else np.asarray(lb_a[a], dtype=np.float64),
        ub=float(book.ub[a]) if ub_a is None else np.asarray(ub_a[a], dtype=np.float64),
        eligible=book.eligible[a],
        gamma=float(book.gamma[a]), kappa=float(book.kappa[a]),
        tau=float(book.tau[a]),
        band_lo=None if not G else book.band_lo[a],
        band_hi=None if not G else book.band_hi[a],
        tax_asset=np.asarray(ta, dtype=np.int64),
        tax_brk=np.asarray(tb, dtype=np.float64).reshape(-1, 3),
        tax_slope=np.asarray(ts, dtype=np.float64).reshape(-1, 4),
        half=uni.half if H else None,
        half_lo=book.half_lo[a] if H else None,
        half_hi=book.half_hi[a] if H else None,
        wb=None if wb is None else wb[a],
        eta=1.0 if eta is None else float(eta[a]),
    )


def box(P: AccountProblem):
    """Per-asset bounds (lb, ub), [0, 0] for excluded assets."""
    lb = np.broadcast_to(np.asarray(P.lb, dtype=np.float64), (P.n,))
    ub = np.broadcast_to(np.asarray(P.ub, dtype=np.float64), (P.n,))
    return np.where(P.eligible, lb, 0.0), np.where(P.eligible, ub, 0.0)


def n_rows(P: AccountProblem) -> int:
    """Constraint rows with two-sided bounds: exposure bands, then the
    policy halfspaces."""
    return P.n_groups + (0 if P.half is None else P.half.shape[0])


def rows_matrix(P: AccountProblem):
    """The (n_rows, n) matrix of those rows: one-hot band rows by group
    label, then the halfspace rows."""
    parts = []
    if P.n_groups:
        A = np.zeros((P.n_groups, P.n))
        A[P.group, np.arange(P.n)] = 1.0
        parts.append(A)
    if P.half is not None:
        parts.append(np.asarray(P.half, dtype=np.float64))
    return np.vstack(parts) if parts else np.zeros((0, P.n))


def rows_bounds(P: AccountProblem):
    """(lo, hi) of the constraint rows, bands first."""
    lo, hi = [], []
    if P.n_groups:
        lo.append(P.band_lo)
        hi.append(P.band_hi)
    if P.half is not None:
        lo.append(P.half_lo)
        hi.append(P.half_hi)
    if not lo:
        return np.zeros(0), np.zeros(0)
    return (np.concatenate(lo).astype(np.float64), np.concatenate(hi).astype(np.float64))


def rows_mul(P: AccountProblem, w):
    """(A w, H w): the constraint rows applied to w (band sums by label,
    then the halfspace rows)."""
    w = np.asarray(w, dtype=np.float64)
    out = []
    if P.n_groups:
        out.append(np.bincount(P.group, weights=w, minlength=P.n_groups))
    if P.half is not None:
        out.append(np.asarray(P.half, dtype=np.float64) @ w)
    return np.concatenate(out) if out else np.zeros(0)


def rows_tmul(P: AccountProblem, lam):
    """A^T lam_band + H^T lam_half for one multiplier per constraint row."""
    lam = np.asarray(lam, dtype=np.float64)
    out = np.zeros(P.n)
    G = P.n_groups
    if G:
        out += lam[:G][P.group]
    if P.half is not None:
        out += np.asarray(P.half, dtype=np.float64).T @ lam[G:]
    return out


def row_coeffs(P: AccountProblem, r: int, idx):
    """Coefficients of constraint row r at the assets idx."""
    G = P.n_groups
    if r < G:
        return (P.group[idx] == r).astype(np.float64)
    return np.asarray(P.half[r - G], dtype=np.float64)[idx]


def linear_term(P: AccountProblem):
    """mu' = eta mu + gamma Sigma w_b: expanding (gamma/2)(w - w_b)^T Sigma
    (w - w_b) - eta mu^T w gives (gamma/2) w^T Sigma w - mu'^T w plus the
    constant (gamma/2) w_b^T Sigma w_b, so the optimum is that of the
    instance without a benchmark and with mu' in place of mu."""
    mu = P.eta * np.asarray(P.mu, dtype=np.float64)
    if P.wb is not None:
        mu = mu + P.gamma * sigma_times(P, np.asarray(P.wb, dtype=np.float64))
    return mu


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


def _active(P: AccountProblem, w):
    w = np.asarray(w, dtype=np.float64)
    return w - P.wb if P.wb is not None else w


def objective(P: AccountProblem, w):
    """f(w) of the build's Eq. 1 instance, recomputed in float64 from its
    definition: (gamma/2)(w - w_b)^T Sigma (w - w_b) - eta mu^T w + trade
    cost."""
    w = np.asarray(w, dtype=np.float64)
    e = _active(P, w)
    return 0.5 * P.gamma * float(e @ sigma_times(P, e)) - P.eta * float(P.mu @ w) \
        + trade_cost(P, w)


def objective_scale(P: AccountProblem, w):
    """Denominator for relative objective errors: |f| or the sum of the
    magnitudes of its terms, whichever is larger (never zero)."""
    w = np.asarray(w, dtype=np.float64)
    e = _active(P, w)
    risk = 0.5 * P.gamma * float(e @ sigma_times(P, e))
    ret = P.eta * float(P.mu @ w)
    tc = trade_cost(P, w)
    return max(abs(risk - ret + tc), risk + abs(ret) + tc, 1e-300)


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
