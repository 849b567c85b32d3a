"""Float64 reference gradients of a linear functional of the optimum
(oracle side; implicit differentiation of the KKT system at w*).

Inside the active pattern of the optimum (fixed coordinates at bounds / kinks,
free coordinates inside a linear piece, binding budget / bands / cap) the
optimum of the build's Eq. 1 instance solves

  gamma Sigma_FF w_F + C_F^T eta = mu_F - slope_F - gamma Sigma_FX w_X
  C_F w_F = h

so w_F is affine in mu and smooth in B.  For L = c^T w:

  [gamma Sigma_FF  C_F^T] [v_F]   [c_F]
  [C_F             0    ] [xi ] = [0  ]      (v = 0 off F)

  dL/dmu = v,
  dL/dB  = -gamma ( v (F B^T w)^T + w (F B^T v)^T ),

the second from d(Sigma w) = dB F B^T w + B F dB^T w on the free rows.  A
coordinate at a kink or bound is held fixed (the generic one-sided
convention; the derivative does not exist where the pattern changes).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .problem import AccountProblem
from .crossover import _classify


def reduced_pattern(P: AccountProblem, w, lam_band, lam_cap, tol=1e-12):
    fixed, val, slope, sgn = _classify(P, w, tol)
    F = np.nonzero(~fixed)[0]
    rows = [np.ones(len(F))]
    G = P.n_groups
    if G:
        Aw = np.bincount(P.group, weights=w, minlength=G)
        for g in range(G):
            at_bound = min(abs(Aw[g] - P.band_hi[g]), abs(Aw[g] - P.band_lo[g])) <= 1e-12
            if at_bound and abs(lam_band[g]) > 0.0:
                rows.append((P.group[F] == g).astype(float))
    if np.isfinite(P.tau) and lam_cap > 0.0:
        rows.append(sgn[F])
    return F, np.vstack(rows)


def gradients(P: AccountProblem, w, lam_band, lam_cap, c):
    """dL/dmu (n,) and dL/dB (n, k) of L = c^T w at the optimum w."""
    F, C = reduced_pattern(P, w, lam_band, lam_cap)
    n, k = P.n, P.k
    dmu = np.zeros(n)
    if len(F):
        BF = P.B[F]
        H = P.gamma * ((BF * P.f) @ BF.T + np.diag(P.d[F]))
        m = C.shape[0]
        K = np.zeros((len(F) + m, len(F) + m))
        K[:len(F), :len(F)] = H
        K[:len(F), len(F):] = C.T
        K[len(F):, :len(F)] = C
        rhs = np.concatenate([c[F], np.zeros(m)])
        sol = np.linalg.lstsq(K, rhs, rcond=1e-14)[0]
        dmu[F] = sol[:len(F)]
    v = dmu
    FBw = P.f * (P.B.T @ w)
    FBv = P.f * (P.B.T @ v)
    dB = -P.gamma * (np.outer(v, FBw) + np.outer(w, FBv))
    return dmu, dB
