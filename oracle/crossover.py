"""Crossover from an interior-point iterate to the exact optimum (oracle).

At the optimum of the build's Eq. 1 instance every eligible coordinate either
sits on a bound / kink of its piecewise-linear trade cost (fixed) or lies
inside one linear piece (free, with a known slope).  Given that classification
and the set of binding constraint rows (bands, halfspaces) and cap, w* solves
one equality-constrained QP:

  gamma (Sigma w)_F - mu'_F + slope_F + lam_cap sgn_F - nu 1 + R_F^T lam = 0
  1^T w = 1,   (R w)_r = bound_r (binding r),   sgn^T (w - w0) = tau (cap)

(mu' = eta mu + gamma Sigma w_b) solved here in float64 (dense for moderate
|F|, factor-space Woodbury otherwise).  The classification is read off the
interior-point iterate with a snap tolerance; several tolerances are tried
and the candidate with the smallest external KKT residual (``oracle.kkt``) is
kept.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .problem import (AccountProblem, kinks_and_slopes, box, n_rows, rows_bounds,
                      rows_mul, row_coeffs, linear_term)
from .kkt import residuals


def _classify(P: AccountProblem, w, tol):
    n = P.n
    fixed = np.zeros(n, dtype=bool)
    val = np.zeros(n)
    slope = np.zeros(n)
    sgn = np.zeros(n)
    taxed = {int(i) for i in P.tax_asset}
    lbv, ubv = box(P)
    for i in range(n):
        lb, ub = lbv[i], ubv[i]
        if not P.eligible[i]:
            fixed[i] = True
            val[i] = 0.0
            continue
        if i in taxed or P.kappa > 0 or np.isfinite(P.tau):
            kinks, slopes = kinks_and_slopes(P, i, 0.0)
        else:
            kinks, slopes = np.zeros(0), np.zeros(1)
        pts = [lb, ub] + [c for c in kinks if lb < c < ub]
        pts = np.asarray(pts)
        dist = np.abs(pts - w[i])
        j = int(np.argmin(dist))
        if dist[j] <= tol:
            fixed[i] = True
            val[i] = pts[j]
        else:
            piece = int(np.searchsorted(kinks, w[i])) if len(kinks) else 0
            slope[i] = slopes[piece]
            sgn[i] = 1.0 if w[i] > P.w0[i] else -1.0
    return fixed, val, slope, sgn


def _solve_reduced(P: AccountProblem, F, rhs, C, h, eta0):
    """Solve [gamma Sigma_FF, C^T; C, 0][w_F; eta] = [rhs; h].

    Eliminating w_F gives S eta = C H^-1 rhs - h with S = C H^-1 C^T.  When
    the free set does not pin every multiplier (an active band with no free
    member, or budget and cap rows parallel on F) S is singular; the system
    is then consistent and the minimum-norm correction of the interior-point
    multipliers eta0 is taken.  w_F does not depend on that choice.
    """
    g = P.gamma
    BF = P.B[F]
    dF = P.d[F]
    nF = len(F)
    if nF == 0:
        return np.zeros(0), np.asarray(eta0, dtype=np.float64)
    if nF <= 3000:
        H = g * ((BF * P.f) @ BF.T + np.diag(dF))
        cho_h = sla.cho_factor(H)

        def Hinv(V):
            return sla.cho_solve(cho_h, V)
    else:
        # Woodbury in factor space: H^-1 = (1/g)(D^-1 - D^-1 B Kf^-1 B^T D^-1)
        Kf = np.diag(1.0 / P.f) + (BF / dF[:, None]).T @ BF
        cho = sla.cho_factor(Kf)

        def Hinv(V):
            V2 = V if V.ndim == 2 else V[:, None]
            DV = V2 / dF[:, None]
            out = (DV - (BF / dF[:, None]) @ sla.cho_solve(cho, BF.T @ DV)) / g
            return out if V.ndim == 2 else out[:, 0]

    Hr = Hinv(rhs)
    HC = Hinv(C.T)
    S = C @ HC
    r = C @ Hr - h
    corr = np.linalg.lstsq(S, r - S @ eta0, rcond=1e-13)[0]
    eta = eta0 + corr
    return Hr - HC @ eta, eta


def _point_slopes(P: AccountProblem, i, x):
    """(lo0, s_lo, hi0, s_hi): the subdifferential of phi_i + lam|.-w0| +
    N_box at the fixed point x is [lo0 + s_lo lam, hi0 + s_hi lam]
    (lo0 = -inf / hi0 = +inf at a bound)."""
    lbv, ubv = box(P)
    lb, ub = lbv[i], ubv[i]
    kinks, slopes = kinks_and_slopes(P, i, 0.0)
    has_phi = P.kappa > 0 or np.isfinite(P.tau) or i in set(int(t) for t in P.tax_asset)
    if not has_phi:
        kinks, slopes = np.zeros(0), np.zeros(1)
    side = lambda q: (-1.0 if q < len(kinks) else 1.0) if len(kinks) else 0.0
    hit = [j for j, c in enumerate(kinks) if c == x]
    if hit:
        j = hit[0]
        lo0, s_lo, hi0, s_hi = slopes[j], side(j), slopes[j + 1], side(j + 1)
    else:
        q = int(np.searchsorted(kinks, x)) if len(kinks) else 0
        lo0, s_lo, hi0, s_hi = slopes[q], side(q), slopes[q], side(q)
    if x <= lb:
        lo0, s_lo = -np.inf, 0.0
    if x >= ub:
        hi0, s_hi = np.inf, 0.0
    return lo0, s_lo, hi0, s_hi


def refine_multipliers(P: AccountProblem, w, fixed, C_rows, act, cap_on, eta,
                       sweeps=3):
    """Move eta = (-nu, band multipliers of the active bands, lam_cap) inside
    the null space of the free-row equations so that every fixed coordinate's
    stationarity interval holds.  Along one null direction n the conditions
    are linear inequalities in the step s; the step is the point of their
    feasible interval nearest to 0 (pulled inside by a small margin).  The
    free-row equations are untouched (C_F^T n = 0)."""
    nc = len(eta)
    if C_rows.shape[1]:
        _, sv, vt = np.linalg.svd(C_rows.T, full_matrices=True)
        rank = int(np.sum(sv > 1e-10 * max(sv.max(), 1.0)))
        N = vt[rank:].T
    else:
        N = np.eye(nc)
    if N.shape[1] == 0:
        return eta
    _, row_hi = rows_bounds(P)
    band_col = {g_: 1 + j for j, (g_, _) in enumerate(act)}
    up = {g_: (bnd == row_hi[g_]) for g_, bnd in act}
    base = P.gamma * (P.B @ (P.f * (P.B.T @ w)) + P.d * w) - linear_term(P)
    rows = [i for i in range(P.n) if fixed[i] and P.eligible[i]]
    geo = {i: _point_slopes(P, i, w[i]) for i in rows}
    idx = np.asarray(rows, dtype=np.int64)
    # coefficients of the active rows at the fixed coordinates
    coef = {g_: dict(zip(rows, row_coeffs(P, g_, idx))) for g_ in band_col}
    for _ in range(sweeps):
        for q in range(N.shape[1]):
            n = N[:, q]
            lam = eta[-1] if cap_on else 0.0
            n_c = n[-1] if cap_on else 0.0
            L, U = -np.inf, np.inf

            def add(alpha, beta):
                nonlocal L, U
                if alpha > 1e-300:
                    U = min(U, beta / alpha)
                elif alpha < -1e-300:
                    L = max(L, beta / alpha)
            for i in rows:
                T = -(base[i] + eta[0])
                a = n[0]
                for g_, col in band_col.items():
                    cf = coef[g_][i]
                    if cf != 0.0:
                        T -= cf * eta[col]
                        a += cf * n[col]
                lo0, s_lo, hi0, s_hi = geo[i]
                if np.isfinite(lo0):      # lo0 + s_lo (lam + s n_c) <= T - a s
                    add(a + s_lo * n_c, T - lo0 - s_lo * lam)
                if np.isfinite(hi0):      # T - a s <= hi0 + s_hi (lam + s n_c)
                    add(-(a + s_hi * n_c), hi0 + s_hi * lam - T)
            if cap_on:                    # lam + s n_c >= 0
                add(-n_c, lam)
            for g_, col in band_col.items():
                if up[g_]:
                    add(-n[col], eta[col])
                else:
                    add(n[col], -eta[col])
            if L <= U:
                s = min(max(0.0, L), U)
                if np.isfinite(L) and np.isfinite(U):
                    mid = 0.5 * (L + U)
                    s = s + 1e-3 * (mid - s)
            else:
                s = 0.5 * (L + U)
            if np.isfinite(s):
                eta = eta + s * n
    return eta


def crossover_once(P: AccountProblem, w, tol, tol_con, nu0=0.0,
                   lam_band0=None, lam_cap0=0.0):
    n = P.n
    fixed, val, slope, sgn = _classify(P, w, tol)
    F = np.nonzero(~fixed)[0]
    X = np.nonzero(fixed)[0]
    wX = val[X]
    G = n_rows(P)
    # binding constraint rows (bands, then halfspaces)
    act = []
    if G:
        row_lo, row_hi = rows_bounds(P)
        Aw = rows_mul(P, w)
        for g_ in range(G):
            if abs(Aw[g_] - row_hi[g_]) <= tol_con:
                act.append((g_, row_hi[g_]))
            elif abs(Aw[g_] - row_lo[g_]) <= tol_con:
                act.append((g_, row_lo[g_]))
    cap_on = bool(np.isfinite(P.tau) and
                  abs(np.abs(w - P.w0).sum() - P.tau) <= tol_con)
    rows, hs = [np.ones(len(F))], [1.0 - wX.sum()]
    for g_, bnd in act:
        rows.append(row_coeffs(P, g_, F))
        hs.append(bnd - float(row_coeffs(P, g_, X) @ wX))
    if cap_on:
        rows.append(sgn[F])
        hs.append(P.tau + float(sgn[F] @ P.w0[F]) -
                  float(np.abs(wX - P.w0[X]).sum()))
    C = np.vstack(rows)
    h = np.asarray(hs)
    # gamma Sigma_FX w_X = gamma B_F F (B_X^T w_X)   (d is diagonal)
    cross = P.gamma * (P.B[F] @ (P.f * (P.B[X].T @ wX))) if len(X) else 0.0
    rhs = linear_term(P)[F] - slope[F] - cross
    eta0 = [-nu0]
    for g_, _ in act:
        eta0.append(0.0 if lam_band0 is None else lam_band0[g_])
    if cap_on:
        eta0.append(lam_cap0)
    wF, eta = _solve_reduced(P, F, rhs, C, h, np.asarray(eta0, float))
    wf = val.copy()
    wf[F] = wF
    eta = refine_multipliers(P, wf, fixed, C, act, cap_on, eta)
    nu = -eta[0]
    lam_band = np.zeros(G)
    for j, (g_, _) in enumerate(act):
        lam_band[g_] = eta[1 + j]
    lam_cap = float(eta[-1]) if cap_on else 0.0
    return wf, (nu, lam_band, lam_cap)


def crossover(P: AccountProblem, w, nu, lam_band, lam_cap,
              tols=(1e-9, 1e-8, 1e-10, 1e-7, 1e-11, 1e-6)):
    """Best of several snap tolerances; falls back to the input point."""
    best = dict(w=np.asarray(w, float), nu=nu, lam_band=lam_band,
                lam_cap=lam_cap, res=residuals(P, w, nu, lam_band, lam_cap),
                method="ipm")
    best_score = max(best["res"]["r_prim"], best["res"]["r_dual"],
                     best["res"]["r_comp"])
    for tol in tols:
        try:
            wf, mult = crossover_once(P, w, tol, max(tol, 1e-9), nu,
                                      lam_band, lam_cap)
        except (np.linalg.LinAlgError, ValueError):
            continue
        if mult is None:
            continue
        r = residuals(P, wf, *mult)
        score = max(r["r_prim"], r["r_dual"], r["r_comp"])
        if score < best_score:
            best = dict(w=wf, nu=mult[0], lam_band=mult[1], lam_cap=mult[2],
                        res=r, method="crossover")
            best_score = score
        if best_score < 1e-13:
            break
    return best
