"""External feasibility and KKT diagnostics (Sec. "External Diagnostics").

Given returned weights and certificate data (nu for the budget, one signed
multiplier per constraint row -- exposure bands, then policy halfspaces --
and lam_cap >= 0 for the turnover cap) this module computes, in float64 and
from the inputs only:

  r_budget   = |1^T w - 1|
  r_box      = max(||(lb - w)_+||_inf, ||(w - ub)_+||_inf)   (excluded: ub = 0)
  r_exposure = max(||(row_lo - R w)_+||_inf, ||(R w - row_hi)_+||_inf), R
               the band rows and the halfspace rows
  r_turnover = (||w - w0||_1 - tau)_+
  r_prim     = max of the four, plus the largest snap distance below

The stationarity check of the paper is written for smooth g_i; the trade costs
here are piecewise linear, so stationarity is checked in its nonsmooth form:
with g = gamma Sigma (w - w_b) - eta mu - nu 1 + R^T lam, every asset must
satisfy -g_i in J_i, the subdifferential of phi_i + lam_cap |. - w0_i| plus
the normal cone of [lb_i, ub_i] at w_i.  A coordinate within eps_snap of a
kink or bound is evaluated at that point; the distance moved is charged to
r_prim.

  r_dual = max_i dist(-g_i, J_i) / scale,  scale = max(||gamma Sigma w||_inf,
           ||mu'||_inf, 1e-12) with mu' = eta mu + gamma Sigma w_b; a negative
           lam_cap is charged here too
  r_comp = max(lam_cap |tau - ||w - w0||_1|, max_r |lam_r| slack_r) / scale

Sign convention for the row multipliers: lam_r > 0 means the upper bound of
row r binds, lam_r < 0 the lower one.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from .problem import (AccountProblem, sigma_times, objective, kinks_and_slopes, box,
                      n_rows, rows_bounds, rows_mul, rows_tmul, linear_term)


def residuals(P: AccountProblem, w, nu, lam_band=None, lam_cap=0.0,
              eps_snap=1e-10):
    w = np.asarray(w, dtype=np.float64)
    n = P.n
    lb, ub = box(P)
    R = n_rows(P)
    lam_band = np.zeros(R) if lam_band is None or R == 0 else \
        np.asarray(lam_band, dtype=np.float64)
    lam_cap = float(lam_cap)

    # ---- primal --------------------------------------------------------
    r_budget = abs(w.sum() - 1.0)
    r_box = max(float(np.max(lb - w, initial=0.0)),
                float(np.max(w - ub, initial=0.0)), 0.0)
    if R:
        row_lo, row_hi = rows_bounds(P)
        Aw = rows_mul(P, w)
        r_exp = max(float(np.max(row_lo - Aw, initial=0.0)),
                    float(np.max(Aw - row_hi, initial=0.0)), 0.0)
    else:
        Aw = np.zeros(0)
        r_exp = 0.0
    turnover = float(np.abs(w - P.w0).sum())
    r_turn = max(turnover - P.tau, 0.0) if np.isfinite(P.tau) else 0.0

    # ---- stationarity --------------------------------------------------
    Sw = sigma_times(P, w)
    mu_eff = linear_term(P)
    grad = P.gamma * Sw - mu_eff
    g = grad - nu
    if R:
        g = g + rows_tmul(P, lam_band)
    target = -g
    lo = np.empty(n)
    hi = np.empty(n)
    snap = np.zeros(n)
    # untaxed assets: one kink at w0 with slopes -/+(kappa + lam_cap)
    kl = P.kappa + lam_cap
    dw = w - P.w0
    at0 = np.abs(dw) <= eps_snap
    lo[:] = np.where(at0, -kl, np.where(dw > 0, kl, -kl))
    hi[:] = np.where(at0, kl, np.where(dw > 0, kl, -kl))
    snap[:] = np.where(at0, np.abs(dw), 0.0)
    # taxed assets: exact piece / kink location
    for i in np.asarray(P.tax_asset, dtype=np.int64):
        kinks, slopes = kinks_and_slopes(P, int(i), lam_cap)
        dist = np.abs(kinks - w[i])
        j = int(np.argmin(dist))
        if dist[j] <= eps_snap:
            lo[i], hi[i] = slopes[j], slopes[j + 1]
            snap[i] = dist[j]
        else:
            piece = int(np.searchsorted(kinks, w[i]))
            lo[i] = hi[i] = slopes[piece]
            snap[i] = 0.0
    # normal cone of [lb, ub]
    at_lb = w <= lb + eps_snap
    at_ub = w >= ub - eps_snap
    snap = np.maximum(snap, np.where(at_lb, np.maximum(w - lb, 0.0), 0.0))
    snap = np.maximum(snap, np.where(at_ub, np.maximum(ub - w, 0.0), 0.0))
    lo = np.where(at_lb, -np.inf, lo)
    hi = np.where(at_ub, np.inf, hi)
    dist = np.maximum(np.maximum(lo - target, target - hi), 0.0)
    scale = max(float(np.max(np.abs(P.gamma * Sw))), float(np.max(np.abs(mu_eff))),
                1e-12)
    r_dual = float(dist.max()) / scale if n else 0.0
    r_dual = max(r_dual, max(-lam_cap, 0.0) / scale)

    # ---- complementarity ----------------------------------------------
    comp = 0.0
    if np.isfinite(P.tau):
        comp = max(comp, max(lam_cap, 0.0) * abs(P.tau - turnover))
    else:
        comp = max(comp, abs(lam_cap))
    if R:
        nz = lam_band != 0.0        # an infinite slack of a one-sided row
        slack = np.where(lam_band > 0, row_hi - Aw, Aw - row_lo)
        comp = max(comp, float(np.max(np.abs(lam_band[nz]) * np.abs(slack[nz]),
                                      initial=0.0)))
    r_comp = comp / scale

    r_prim = max(r_budget, r_box, r_exp, r_turn) + float(snap.max(initial=0.0))
    return dict(r_prim=r_prim, r_dual=r_dual, r_comp=r_comp,
                r_budget=r_budget, r_box=r_box, r_exposure=r_exp,
                r_turnover=r_turn, obj=objective(P, w), scale=scale,
                turnover=turnover)
