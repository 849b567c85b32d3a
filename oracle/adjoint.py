"""Float64 reference gradients of a linear functional of the optimum
(oracle side; implicit differentiation of the KKT system at w*).

Inside the active pattern of the optimum (fixed coordinates at bounds / kinks,
free coordinates inside a linear piece, binding budget / constraint rows /
cap) the optimum of the build's Eq. 1 instance solves

  gamma Sigma_FF w_F + C_F^T eta = mu'_F - slope_F - gamma Sigma_FX w_X
  C_F w_F = h,        mu' = eta mu + gamma Sigma w_b,

so w_F is affine in mu and smooth in B.  For L = c^T w:

  [gamma Sigma_FF  C_F^T] [v_F]   [c_F]
  [C_F             0    ] [xi ] = [0  ]      (v = 0 off F)

  dL/dmu = eta v,
  dL/dB  = -gamma ( v (F B^T e)^T + e (F B^T v)^T ),   e = w - w_b,

the second from d(Sigma e) = dB F B^T e + B F dB^T e on the free rows (the
risk term is (gamma/2) e^T Sigma e; the constraint rows are data of their
own and do not move with B).  A coordinate at a kink or bound is held fixed
(the generic one-sided convention; the derivative does not exist where the
pattern changes).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .problem import AccountProblem, n_rows, rows_bounds, rows_mul, row_coeffs
from .crossover import _classify


def reduced_pattern(P: AccountProblem, w, lam_band, lam_cap, tol=1e-12):
    fixed, val, slope, sgn = _classify(P, w, tol)
    F = np.nonzero(~fixed)[0]
    rows = [np.ones(len(F))]
    G = n_rows(P)
    if G:
        row_lo, row_hi = rows_bounds(P)
        Aw = rows_mul(P, w)
        for g in range(G):
            at_bound = min(abs(Aw[g] - row_hi[g]), abs(Aw[g] - row_lo[g])) <= 1e-12
            if at_bound and abs(lam_band[g]) > 0.0:
                rows.append(row_coeffs(P, g, F))
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
    e = w - P.wb if P.wb is not None else w
    FBe = P.f * (P.B.T @ e)
    FBv = P.f * (P.B.T @ v)
    dB = -P.gamma * (np.outer(v, FBe) + np.outer(e, FBv))
    return P.eta * dmu, dB
