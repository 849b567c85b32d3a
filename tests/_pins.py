"""Independent reference constructions that pin the oracle.

Nothing here imports ``oracle``: each function restates the mathematics of
the build's Eq. 1 instance (paper Sec. "Benchmark Problem Class") in the most
direct way available for a special case.

  closed_form_budget_only   Eq. 1 with only the budget row: stationarity
                            gamma Sigma w - mu - nu 1 = 0 solved with a dense
                            Sigma, w = Sigma^-1 (mu + nu 1) / gamma
  brute_force               every active-set pattern of a tiny instance
                            enumerated, each equality QP solved densely, the
                            one satisfying all KKT conditions returned
  separable_exact           Sigma diagonal (B = 0): each coordinate's 1-D
                            problem is solved by evaluating every candidate
                            point, and the budget / cap multipliers are found
                            by nested bisection (monotone in each)
"""
from __future__ import annotations

import itertools

import numpy as np


# ---------------------------------------------------------------------------
# dense problem pieces
# ---------------------------------------------------------------------------
def dense_sigma(B, f, d):
    return (B * f) @ B.T + np.diag(d)


def phi_pieces(w0, kappa, brk=None, slope=None):
    """Kinks (ascending) and slopes of kappa|w - w0| + T((w0 - w)_+)."""
    if brk is None:
        return np.array([w0]), np.array([-kappa, kappa])
    kinks = np.array([w0 - brk[2], w0 - brk[1], w0 - brk[0], w0])
    slopes = -kappa - np.array([slope[3], slope[2], slope[1], slope[0]])
    return kinks, np.append(slopes, kappa)


def phi_value(w, w0, kappa, brk=None, slope=None):
    """Direct evaluation: kappa |dw| + integral of the lot slopes over the
    sold amount (lots consumed in order)."""
    dw = w - w0
    v = kappa * abs(dw)
    if brk is not None and dw < 0:
        sold = -dw
        edges = [0.0, brk[0], brk[1], brk[2], np.inf]
        for j in range(4):
            take = min(max(sold - edges[j], 0.0), edges[j + 1] - edges[j])
            v += slope[j] * take
    return v


# ---------------------------------------------------------------------------
# closed form
# ---------------------------------------------------------------------------
def closed_form_budget_only(B, f, d, mu, gamma):
    """min (gamma/2) w^T Sigma w - mu^T w  s.t. 1^T w = 1."""
    S = dense_sigma(B, f, d)
    one = np.ones(len(mu))
    Si_mu = np.linalg.solve(S, mu)
    Si_1 = np.linalg.solve(S, one)
    nu = (gamma - one @ Si_mu) / (one @ Si_1)
    w = (Si_mu + nu * Si_1) / gamma
    return w, nu


def closed_form_benchmark(B, f, d, mu, gamma, wb, eta):
    """min (gamma/2)(w - wb)^T Sigma (w - wb) - eta mu^T w  s.t. 1^T w = 1:
    stationarity gamma Sigma (w - wb) - eta mu - nu 1 = 0, so
    w = wb + Sigma^-1 (eta mu + nu 1) / gamma with nu from the budget."""
    S = dense_sigma(B, f, d)
    one = np.ones(len(mu))
    Si_mu = np.linalg.solve(S, eta * mu)
    Si_1 = np.linalg.solve(S, one)
    nu = (gamma * (1.0 - one @ wb) - one @ Si_mu) / (one @ Si_1)
    w = wb + (Si_mu + nu * Si_1) / gamma
    return w, nu


# ---------------------------------------------------------------------------
# brute-force active-set enumeration (tiny N)
# ---------------------------------------------------------------------------
def brute_force(B, f, d, mu, gamma, lb, ub, w0=None, kappa=0.0, tax=None,
                group=None, band_lo=None, band_hi=None, tau=np.inf,
                tol=1e-9, half=None, half_lo=None, half_hi=None, wb=None,
                eta=1.0):
    """Enumerate, per asset, 'at point p' / 'inside piece q' states (points:
    bounds and kinks of the trade cost inside the box), per constraint row
    (band by group label, or dense halfspace row) off / at-lo / at-hi (an
    infinite bound has no 'at' state), and cap off / on.  Each pattern gives
    a linear system; a pattern is accepted when its solution lies in the
    stated pieces, satisfies every inactive constraint, and its multipliers
    have the right signs and lie in the subdifferential at fixed
    coordinates.  lb / ub may be per-asset arrays; the objective is
    (1/2)(w - wb)^T (gamma Sigma) (w - wb) - eta mu^T w + trade cost, whose
    gradient gamma Sigma (w - wb) - eta mu enters the stationarity rows.

    Returns (w, nu, lam_rows, lam_cap, n_accepted), lam_rows bands first.
    """
    n = len(mu)
    S = gamma * dense_sigma(B, f, d)
    w0 = np.zeros(n) if w0 is None else w0
    tax = tax or {}
    has_phi = kappa > 0 or bool(tax) or np.isfinite(tau)
    lbv = np.broadcast_to(np.asarray(lb, dtype=np.float64), (n,))
    ubv = np.broadcast_to(np.asarray(ub, dtype=np.float64), (n,))
    # constraint rows: one-hot bands, then dense halfspace rows
    rows, rlo, rhi = [], [], []
    if group is not None:
        for g in range(int(band_lo.shape[0])):
            rows.append((np.asarray(group) == g).astype(float))
            rlo.append(band_lo[g])
            rhi.append(band_hi[g])
    if half is not None:
        for h in range(half.shape[0]):
            rows.append(np.asarray(half[h], dtype=np.float64))
            rlo.append(half_lo[h])
            rhi.append(half_hi[h])
    G = len(rows)
    Rm = np.vstack(rows) if G else np.zeros((0, n))
    grad0 = -eta * np.asarray(mu, dtype=np.float64)
    if wb is not None:
        grad0 = grad0 - S @ wb

    per_asset = []
    for i in range(n):
        if has_phi:
            t = tax.get(i)
            kinks, slopes = phi_pieces(w0[i], kappa, *(t if t else (None, None)))
        else:
            kinks, slopes = np.zeros(0), np.zeros(1)
        lb, ub = lbv[i], ubv[i]
        pts = [lb, ub] + [c for c in kinks if lb < c < ub]
        pts = sorted(set(pts))
        states = [("at", p) for p in pts]
        for a_, b_ in zip(pts[:-1], pts[1:]):
            mid = 0.5 * (a_ + b_)
            q = int(np.searchsorted(kinks, mid)) if len(kinks) else 0
            sgn = 1.0 if mid > w0[i] else -1.0
            states.append(("in", (a_, b_, slopes[q], sgn)))
        per_asset.append((states, kinks, slopes))

    band_states = list(itertools.product(*[
        ["off"] + (["lo"] if np.isfinite(rlo[g]) else []) + (["hi"] if np.isfinite(rhi[g]) else [])
        for g in range(G)]))
    cap_states = ("off", "on") if np.isfinite(tau) else ("off",)

    def subdiff(i, x, lam_cap):
        """Interval of d/dw [phi_i + lam_cap |w - w0_i|] + N_box at x."""
        _, kinks, slopes = per_asset[i]
        if len(kinks):
            # w0 is always the last kink: pieces left of it are sales (-lam),
            # the last piece is the buy side (+lam)
            sl = slopes + np.where(np.arange(len(slopes)) < len(kinks),
                                   -lam_cap, lam_cap)
            j = [m for m, c in enumerate(kinks) if abs(c - x) <= tol]
            if j:
                lo_, hi_ = sl[j[0]], sl[j[0] + 1]
            else:
                q = int(np.searchsorted(kinks, x))
                lo_ = hi_ = sl[q]
        else:
            lo_ = hi_ = 0.0
        if abs(x - lbv[i]) <= tol:
            lo_ = -np.inf
        if abs(x - ubv[i]) <= tol:
            hi_ = np.inf
        return lo_, hi_

    found = []
    for combo in itertools.product(*[s for s, _, _ in per_asset]):
        for bst in band_states:
            for cst in cap_states:
                # unknowns: w (n), nu, lam_g (active), lam_cap
                act = [g for g in range(G) if bst[g] != "off"]
                m = n + 1 + len(act) + (1 if cst == "on" else 0)
                M = np.zeros((m, m))
                r = np.zeros(m)
                sgn_all = np.zeros(n)
                for i, st in enumerate(combo):
                    if st[0] == "at":
                        M[i, i] = 1.0
                        r[i] = st[1]
                        sgn_all[i] = np.sign(st[1] - w0[i])
                    else:
                        M[i, :n] = S[i]
                        M[i, n] = -1.0
                        r[i] = -grad0[i] - st[1][2]
                        sgn_all[i] = st[1][3]
                for j, g in enumerate(act):
                    for i, st in enumerate(combo):
                        if st[0] == "in":
                            M[i, n + 1 + j] = Rm[g, i]
                if cst == "on":
                    for i, st in enumerate(combo):
                        if st[0] == "in":
                            M[i, m - 1] = st[1][3]
                row = n
                M[row, :n] = 1.0
                r[row] = 1.0
                for j, g in enumerate(act):
                    M[n + 1 + j, :n] = Rm[g]
                    r[n + 1 + j] = rlo[g] if bst[g] == "lo" else rhi[g]
                if cst == "on":
                    M[m - 1, :n] = sgn_all
                    r[m - 1] = tau + sgn_all @ w0
                try:
                    sol = np.linalg.solve(M, r)
                except np.linalg.LinAlgError:
                    continue
                w = sol[:n]
                nu = sol[n]
                lam = np.zeros(G)
                for j, g in enumerate(act):
                    lam[g] = sol[n + 1 + j]
                lam_cap = sol[m - 1] if cst == "on" else 0.0
                ok = True
                # pieces and bounds
                for i, st in enumerate(combo):
                    if st[0] == "in":
                        a_, b_ = st[1][0], st[1][1]
                        if not (a_ - tol <= w[i] <= b_ + tol):
                            ok = False
                            break
                if not ok:
                    continue
                # inactive constraints, signs
                if G:
                    Aw = Rm @ w
                    for g in range(G):
                        if bst[g] == "off" and not (rlo[g] - tol <= Aw[g]
                                                    <= rhi[g] + tol):
                            ok = False
                        if bst[g] == "hi" and lam[g] < -tol:
                            ok = False
                        if bst[g] == "lo" and lam[g] > tol:
                            ok = False
                if cst == "off" and np.isfinite(tau) and \
                        np.abs(w - w0).sum() > tau + tol:
                    ok = False
                if cst == "on" and lam_cap < -tol:
                    ok = False
                if not ok:
                    continue
                # subgradient condition at fixed coordinates
                grad = S @ w + grad0 - nu
                if G:
                    grad = grad + Rm.T @ lam
                for i, st in enumerate(combo):
                    if st[0] == "at":
                        lo_, hi_ = subdiff(i, w[i], lam_cap)
                        if not (lo_ - 1e-9 <= -grad[i] <= hi_ + 1e-9):
                            ok = False
                            break
                if ok:
                    found.append((w, nu, lam, lam_cap))
    if not found:
        raise RuntimeError("no KKT pattern found")
    w = found[0][0]
    for other in found[1:]:
        if np.max(np.abs(other[0] - w)) > 1e-7:
            raise RuntimeError("two different KKT points (not convex?)")
    return found[0][0], found[0][1], found[0][2], found[0][3], len(found)


# ---------------------------------------------------------------------------
# separable problem (B = 0): nested bisection
# ---------------------------------------------------------------------------
def _coord_min(q, lin, lb, ub, kinks, slopes):
    """argmin over [lb, ub] of (q/2) x^2 - lin x + pwl(x), pwl given by kinks
    and slopes (value 0 at the first kink or at lb): evaluate every candidate
    (bounds, kinks inside, stationary point of each piece clipped to it)."""
    def pwl(x):
        if len(kinks) == 0:
            return 0.0
        v = 0.0
        # integrate slope from kinks[0] to x
        pts = np.concatenate([[-np.inf], kinks, [np.inf]])
        ref = kinks[0]
        if x >= ref:
            for j in range(1, len(pts) - 1):
                a_, b_ = pts[j], pts[j + 1]
                if x > a_:
                    v += slopes[j] * (min(x, b_) - a_)
        else:
            v += -slopes[0] * (ref - x)
        return v

    cands = [lb, ub] + [c for c in kinks if lb < c < ub]
    edges = np.concatenate([[-np.inf], kinks, [np.inf]])
    for j in range(len(slopes)):
        x = (lin - slopes[j]) / q
        x = min(max(x, edges[j]), edges[j + 1])
        x = min(max(x, lb), ub)
        cands.append(x)
    vals = [0.5 * q * x * x - lin * x + pwl(x) for x in cands]
    return cands[int(np.argmin(vals))]


def _untaxed_min(q, lin, lb, ub, w0, s):
    """Vectorised argmin over [lb, ub] of (q/2)x^2 - lin x + s|x - w0| by
    comparing the objective at every candidate: both bounds, the kink w0
    (when inside) and the stationary point of each side clipped to it."""
    big = np.inf
    cands = [np.full_like(lin, lb), np.full_like(lin, ub),
             np.clip(w0, lb, ub),
             np.clip(np.maximum((lin - s) / q, w0), lb, ub),
             np.clip(np.minimum((lin + s) / q, w0), lb, ub)]
    vals = [0.5 * q * x * x - lin * x + s * np.abs(x - w0) for x in cands]
    vals = np.where(np.isfinite(vals), vals, big)
    best = np.argmin(np.vstack(vals), axis=0)
    return np.choose(best, cands)


def separable_exact(d, mu, gamma, lb, ub, eligible, w0, kappa, tax, tau,
                    iters=100):
    """Sigma = diag(d).  w_i(nu, lam) minimises its own 1-D problem; the
    budget multiplier nu (sum w increasing in nu) and cap multiplier lam
    (turnover decreasing in lam) are found by bisection."""
    n = len(mu)
    tax = tax or {}
    taxed = np.array(sorted(tax), dtype=np.int64)
    plain = np.ones(n, dtype=bool)
    plain[taxed] = False
    plain &= eligible

    def w_of(nu, lam):
        w = np.zeros(n)
        w[plain] = _untaxed_min(gamma * d[plain], mu[plain] + nu, lb, ub,
                                w0[plain], kappa + lam)
        for i in taxed:
            if not eligible[i]:
                continue
            kinks, slopes = phi_pieces(w0[i], kappa, *tax[i])
            slopes = slopes + np.where(np.arange(len(slopes)) < len(kinks),
                                       -lam, lam)
            w[i] = _coord_min(gamma * d[i], mu[i] + nu, lb, ub, kinks, slopes)
        return w

    def solve_nu(lam):
        lo, hi = -1.0, 1.0
        while w_of(lo, lam).sum() > 1.0:
            lo *= 2
        while w_of(hi, lam).sum() < 1.0:
            hi *= 2
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if mid == lo or mid == hi:
                break
            if w_of(mid, lam).sum() < 1.0:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    nu = solve_nu(0.0)
    w = w_of(nu, 0.0)
    if not np.isfinite(tau) or np.abs(w - w0).sum() <= tau:
        return w, nu, 0.0
    lo, hi = 0.0, 1.0
    while np.abs(w_of(solve_nu(hi), hi) - w0).sum() > tau:
        hi *= 2
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if np.abs(w_of(solve_nu(mid), mid) - w0).sum() > tau:
            lo = mid
        else:
            hi = mid
    lam = 0.5 * (lo + hi)
    nu = solve_nu(lam)
    return w_of(nu, lam), nu, lam
