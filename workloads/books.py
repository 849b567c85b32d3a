"""Seeded synthetic universes and books of accounts.

The shapes and value distributions follow the batched-rebalancing workload of
the paper (Sec. "Public Benchmark Workload", the batched account rebalancing
collection and the problem class of Eq. 1) at the five sizes used throughout
this project:

  c1  1 account,   N=100,     k=5,   budget + long-only box [0, 0.1]
  c2  64 accounts, N=2,000,   k=40,  box [0, 0.05], 10 sector bands (+/-0.05
      absolute around the sector's share of names), L1 turnover 1e-3|w-w0|,
      w0 ~ Dirichlet(1)
  c3  500 accounts, N=10,000, k=80,  box [0, 0.01], exclusion masks leaving a
      U[0.3,1] fraction eligible, 100-400 held names, 4-lot piecewise-linear
      tax on sales, turnover cap tau = tau_min + 0.1
  c4  128 accounts, N=5,000,  k=60,  as c2 with box [0, 0.02], gamma = 1000
  c5  8 accounts, N=384,800,  k=100, 50 one-hot groups (+/-0.005), box
      [0, 1e-3], L1 turnover 1e-3, 2,000 held names with 4-lot tax
  e7  200 accounts, N=481,   k=20,  box [0, 0.03], L1 transition cost
      5e-3|w-w0|, drifted holdings w0 ~ Dirichlet(1): the shape of the
      paper's small-universe batch scenario on its real 481-name universe

The paper's own instances (real S&P 500 data, Sec. "Operationally Constrained
Real-Data Scenarios") are not available; these synthetic books stand in for
them.  Every floating-point value is rounded to float32 and stored as float64,
so a float32 device path and the float64 oracle see exactly the same problem.

Universe draws: B ~ N(0, 0.1^2), f ~ U[0.01, 0.05], d ~ U[1e-4, 1e-3].
Account draws: mu ~ N(5e-4, sd 1e-2), one generator per account spawned from
SeedSequence([config id, seed]) so that an account's data does not depend on
how many accounts are drawn.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5", "e7")
_CFG_ID = {name: i for i, name in enumerate(CONFIG_NAMES)}


def to_f32_exact(x):
    """Round to float32 and return float64 holding exactly those values."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclass
class Universe:
    """Factor-model universe shared by every account of a book.

    Sigma = B diag(f) B^T + diag(d).  ``group`` holds one label per asset in
    [0, n_groups) (one-hot exposure rows) or is None when there are no bands.
    """
    B: np.ndarray            # (N, k)
    f: np.ndarray            # (k,)
    d: np.ndarray            # (N,)
    group: Optional[np.ndarray] = None   # (N,) int32
    n_groups: int = 0
    # policy halfspace rows of Eq. 1 shared by the book (for example factor
    # exposures B[:, j]^T w); each account bounds them with half_lo/half_hi
    half: Optional[np.ndarray] = None    # (H, N)

    @property
    def n_half(self) -> int:
        return 0 if self.half is None else self.half.shape[0]

    @property
    def n(self) -> int:
        return self.B.shape[0]

    @property
    def k(self) -> int:
        return self.B.shape[1]


@dataclass
class Book:
    """Per-account data of Eq. 1 for M accounts over one universe.

    Lot data for the sale-side tax is CSR over accounts: entries
    tax_ptr[a]:tax_ptr[a+1] belong to account a, sorted by asset.  Breakpoints
    are cumulative sale amounts 0 < b1 < b2 < b3; slopes s0 <= s1 <= s2 <= s3
    are the marginal tax per unit sold inside each lot (the last one also
    applies beyond b3).
    """
    mu: np.ndarray           # (M, N)
    w0: np.ndarray           # (M, N)
    lb: np.ndarray           # (M,)
    ub: np.ndarray           # (M,)
    eligible: np.ndarray     # (M, N) bool
    gamma: np.ndarray        # (M,)
    kappa: np.ndarray        # (M,)
    tau: np.ndarray          # (M,)  +inf = no cap
    band_lo: Optional[np.ndarray] = None   # (M, G)
    band_hi: Optional[np.ndarray] = None   # (M, G)
    tax_ptr: np.ndarray = field(default_factory=lambda: np.zeros(1, np.int64))
    tax_asset: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    tax_brk: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    tax_slope: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    # the rest of Eq. 1 (all optional): per-asset bounds (replacing lb / ub
    # for eligible names), bounds of the universe's halfspace rows (-inf /
    # +inf: one-sided), benchmark weights w_b and the return scale eta
    lb_asset: Optional[np.ndarray] = None  # (M, N)
    ub_asset: Optional[np.ndarray] = None  # (M, N)
    half_lo: Optional[np.ndarray] = None   # (M, H)
    half_hi: Optional[np.ndarray] = None   # (M, H)
    wb: Optional[np.ndarray] = None        # (M, N)
    eta: Optional[np.ndarray] = None       # (M,)

    @property
    def m(self) -> int:
        return self.mu.shape[0]

    @property
    def n(self) -> int:
        return self.mu.shape[1]

    def tax_of(self, a: int):
        """(assets, breakpoints, slopes) of account a."""
        s, e = int(self.tax_ptr[a]), int(self.tax_ptr[a + 1])
        return self.tax_asset[s:e], self.tax_brk[s:e], self.tax_slope[s:e]


# --------------------------------------------------------------------------
# defaults per configuration
# --------------------------------------------------------------------------
_DEFAULTS = {
    "c1": dict(N=100, M=1, k=5, ub=0.1, gamma=1.0, kappa=0.0, groups=0,
               band_halfwidth=None, elig=(1.0, 1.0), held=None, tax=False,
               cap_slack=None),
    "c2": dict(N=2000, M=64, k=40, ub=0.05, gamma=1.0, kappa=1e-3, groups=10,
               band_halfwidth=0.05, elig=(1.0, 1.0), held=None, tax=False,
               cap_slack=None),
    "c3": dict(N=10000, M=500, k=80, ub=0.01, gamma=1.0, kappa=0.0, groups=0,
               band_halfwidth=None, elig=(0.3, 1.0), held=(100, 400), tax=True,
               cap_slack=0.1),
    "c4": dict(N=5000, M=128, k=60, ub=0.02, gamma=1000.0, kappa=1e-3,
               groups=10, band_halfwidth=0.05, elig=(1.0, 1.0), held=None,
               tax=False, cap_slack=None),
    "c5": dict(N=384800, M=8, k=100, ub=1e-3, gamma=1.0, kappa=1e-3,
               groups=50, band_halfwidth=0.005, elig=(1.0, 1.0),
               held=(2000, 2000), tax=True, cap_slack=None),
    "e7": dict(N=481, M=200, k=20, ub=0.03, gamma=1.0, kappa=5e-3, groups=0,
               band_halfwidth=None, elig=(1.0, 1.0), held=None, tax=False,
               cap_slack=None),
}


def config_defaults(name: str) -> dict:
    return dict(_DEFAULTS[name])


def _project_capped_simplex(v, cap, total=1.0):
    """Euclidean projection of v onto {0 <= x <= cap, sum x = total} by
    bisection on the shift (input construction only)."""
    lo, hi = v.min() - cap - 1.0, v.max() + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = np.clip(v - mid, 0.0, cap).sum()
        if s > total:
            lo = mid
        else:
            hi = mid
    return np.clip(v - 0.5 * (lo + hi), 0.0, cap)


def _make_universe(rng, N, k, groups):
    B = to_f32_exact(rng.normal(0.0, 0.1, size=(N, k)))
    f = to_f32_exact(rng.uniform(0.01, 0.05, size=k))
    d = to_f32_exact(rng.uniform(1e-4, 1e-3, size=N))
    group = None
    if groups:
        group = rng.integers(0, groups, size=N).astype(np.int32)
    return Universe(B=B, f=f, d=d, group=group, n_groups=int(groups))


def _strictly_increasing_f32(b, top):
    """Make float32 breakpoints strictly increasing and below ``top``."""
    b = to_f32_exact(b)
    for j in range(1, len(b)):
        if b[j] <= b[j - 1]:
            b[j] = float(np.nextafter(np.float32(b[j - 1]), np.float32(np.inf)))
    return b


def make_config(name: str, seed: int = 0, **over) -> tuple[Universe, Book]:
    """Draw the universe and book of configuration ``name`` (c1..c5).

    Keyword overrides (N, M, k, ub, gamma, kappa, groups, band_halfwidth, elig,
    held, tax, cap_slack, mu_mean, mu_sd, w0) scale a configuration down for
    tests or switch features on and off.  ``w0='dirichlet'`` forces a dense
    Dirichlet(1) starting portfolio; ``w0='zero'`` forces an empty one.

    The rest of Eq. 1, off by default: ``halfspaces=H`` adds H policy rows,
    the exposures to the first H factors, bounded within
    ``half_halfwidth`` of the equal-weight exposure (the last row one-sided,
    upper bound only); ``asset_bounds=True`` draws per-asset upper bounds
    ub * U[0.5, 1.5] and a minimum holding of a fifth of that on 2 % of the
    eligible names; ``benchmark=True`` draws benchmark weights w_b (a
    Dirichlet portfolio projected onto the box) and eta ~ U[0.5, 1.5].
    These draws come after every other draw of the account, so switching
    them on leaves the rest of the book unchanged.
    """
    p = config_defaults(name)
    p.update(mu_mean=5e-4, mu_sd=1e-2, w0=None, halfspaces=0, half_halfwidth=2e-3,
             asset_bounds=False, benchmark=False)
    for key, val in over.items():
        if key not in p:
            raise KeyError(f"unknown override {key!r}")
        p[key] = val
    N, M, k = int(p["N"]), int(p["M"]), int(p["k"])
    ss = np.random.SeedSequence([_CFG_ID[name], int(seed)])
    kids = ss.spawn(M + 1)
    uni = _make_universe(np.random.default_rng(kids[0]), N, k, int(p["groups"]))

    G = uni.n_groups
    ub = float(p["ub"])
    mu = np.empty((M, N))
    w0 = np.zeros((M, N))
    elig = np.ones((M, N), dtype=bool)
    tau = np.full(M, np.inf)
    band_lo = band_hi = None
    if G:
        share = np.bincount(uni.group, minlength=G) / N
        hw = float(p["band_halfwidth"])
        band_lo = np.tile(to_f32_exact(np.maximum(share - hw, 0.0)), (M, 1))
        band_hi = np.tile(to_f32_exact(share + hw), (M, 1))
    t_ptr = [0]
    t_asset, t_brk, t_slope = [], [], []
    H = int(p["halfspaces"])
    if H > k:
        raise ValueError("halfspaces: at most one row per factor")
    half = half_lo = half_hi = None
    if H:
        half = np.ascontiguousarray(uni.B[:, :H].T)
        uni = replace(uni, half=half)
        ew = half.sum(axis=1) / N
        hw = float(p["half_halfwidth"])
        half_lo = np.tile(to_f32_exact(ew - hw), (M, 1))
        half_hi = np.tile(to_f32_exact(ew + hw), (M, 1))
        half_lo[:, H - 1] = -np.inf
    lb_asset = np.zeros((M, N)) if p["asset_bounds"] else None
    ub_asset = np.zeros((M, N)) if p["asset_bounds"] else None
    wb = np.zeros((M, N)) if p["benchmark"] else None
    eta = np.ones(M) if p["benchmark"] else None

    w0_mode = p["w0"]
    if w0_mode is None:
        w0_mode = "held" if p["held"] is not None else "dirichlet"

    for a in range(M):
        rng = np.random.default_rng(kids[a + 1])
        mu[a] = to_f32_exact(rng.normal(p["mu_mean"], p["mu_sd"], size=N))
        lo_frac, hi_frac = p["elig"]
        if lo_frac < 1.0:
            frac = rng.uniform(lo_frac, hi_frac)
            n_e = int(math.ceil(frac * N))
            mask = np.zeros(N, dtype=bool)
            mask[rng.choice(N, size=n_e, replace=False)] = True
            elig[a] = mask
        if w0_mode == "dirichlet":
            w0[a] = to_f32_exact(rng.dirichlet(np.ones(N)))
        elif w0_mode == "held":
            h_lo, h_hi = p["held"]
            n_h = int(rng.integers(h_lo, h_hi + 1))
            n_h = min(n_h, N)
            idx = np.sort(rng.choice(N, size=n_h, replace=False))
            raw = rng.dirichlet(np.ones(n_h))
            cap = max(ub, 1.0 / n_h)
            w0[a, idx] = to_f32_exact(_project_capped_simplex(raw, cap))
        elif w0_mode == "zero":
            pass
        else:
            raise ValueError(w0_mode)
        if p["tax"]:
            held = np.nonzero(w0[a] > 0)[0]
            for i in held:
                fr = rng.dirichlet(np.ones(4))
                brk = np.cumsum(fr)[:3] * w0[a, i]
                brk = _strictly_increasing_f32(brk, w0[a, i])
                slope = to_f32_exact(np.sort(rng.uniform(0.0, 5e-3, size=4)))
                t_asset.append(i)
                t_brk.append(brk)
                t_slope.append(slope)
        t_ptr.append(len(t_asset))
        if p["asset_bounds"]:
            ub_asset[a] = to_f32_exact(ub * rng.uniform(0.5, 1.5, size=N))
            n_min = int(0.02 * np.count_nonzero(elig[a]))
            pick = rng.choice(np.nonzero(elig[a])[0], size=n_min, replace=False)
            lb_asset[a, pick] = to_f32_exact(0.2 * ub_asset[a, pick])
        if p["benchmark"]:
            cap_b = ub_asset[a] if p["asset_bounds"] else np.full(N, ub)
            raw = rng.dirichlet(np.ones(N))
            wb[a] = to_f32_exact(np.minimum(_project_capped_simplex(raw, float(cap_b.max())),
                                            cap_b))
            eta[a] = to_f32_exact(rng.uniform(0.5, 1.5))
        if p["cap_slack"] is not None:
            u_a = np.where(elig[a], ub_asset[a] if p["asset_bounds"] else ub, 0.0)
            tau_min = 2.0 * np.maximum(w0[a] - u_a, 0.0).sum()
            t = np.float32(tau_min + float(p["cap_slack"]))
            tau[a] = float(t)

    book = Book(
        mu=mu, w0=w0,
        lb=np.zeros(M), ub=np.full(M, to_f32_exact(ub)),
        eligible=elig,
        gamma=np.full(M, to_f32_exact(p["gamma"])),
        kappa=np.full(M, to_f32_exact(p["kappa"])),
        tau=tau, band_lo=band_lo, band_hi=band_hi,
        tax_ptr=np.asarray(t_ptr, dtype=np.int64),
        tax_asset=np.asarray(t_asset, dtype=np.int32).reshape(-1),
        tax_brk=np.asarray(t_brk, dtype=np.float64).reshape(-1, 3),
        tax_slope=np.asarray(t_slope, dtype=np.float64).reshape(-1, 4),
        lb_asset=lb_asset, ub_asset=ub_asset, half_lo=half_lo, half_hi=half_hi,
        wb=wb, eta=eta,
    )
    return uni, book


def subset_accounts(book: Book, idx) -> Book:
    """Book restricted to the accounts ``idx`` (in that order)."""
    idx = np.asarray(idx, dtype=np.int64).reshape(-1)
    ptr, assets, brk, slope = [0], [], [], []
    for a in idx:
        s, e = int(book.tax_ptr[a]), int(book.tax_ptr[a + 1])
        assets.append(book.tax_asset[s:e])
        brk.append(book.tax_brk[s:e])
        slope.append(book.tax_slope[s:e])
        ptr.append(ptr[-1] + e - s)
    cat = (lambda xs, shape: np.concatenate(xs) if xs else np.zeros(shape))
    return replace(
        book,
        mu=book.mu[idx].copy(), w0=book.w0[idx].copy(),
        lb=book.lb[idx].copy(), ub=book.ub[idx].copy(),
        eligible=book.eligible[idx].copy(),
        gamma=book.gamma[idx].copy(), kappa=book.kappa[idx].copy(),
        tau=book.tau[idx].copy(),
        band_lo=None if book.band_lo is None else book.band_lo[idx].copy(),
        band_hi=None if book.band_hi is None else book.band_hi[idx].copy(),
        tax_ptr=np.asarray(ptr, dtype=np.int64),
        tax_asset=cat(assets, (0,)).astype(np.int32),
        tax_brk=cat(brk, (0, 3)).reshape(-1, 3),
        tax_slope=cat(slope, (0, 4)).reshape(-1, 4),
        lb_asset=None if book.lb_asset is None else book.lb_asset[idx].copy(),
        ub_asset=None if book.ub_asset is None else book.ub_asset[idx].copy(),
        half_lo=None if book.half_lo is None else book.half_lo[idx].copy(),
        half_hi=None if book.half_hi is None else book.half_hi[idx].copy(),
        wb=None if book.wb is None else book.wb[idx].copy(),
        eta=None if book.eta is None else book.eta[idx].copy(),
    )
