"""Float64 primal-dual interior-point solver for one account (oracle).

The paper's engine is closed (Sec. "Claim Boundary"), so the oracle does not
follow any published listing: it solves the convex program of Eq. 1 (Sec.
"Benchmark Problem Class"), as instantiated in ``oracle.problem``, with a
textbook Mehrotra predictor-corrector method on an equivalent lifted QP whose
Hessian is diagonal:

  variables  w_i (eligible assets), y = B^T w (k), buys p_i >= 0, sales
             s_ij >= 0 split into tax lots (0 <= s_ij <= lot length, the last
             lot unbounded), row values t_r in [row_lo, row_hi] (exposure
             bands, then policy halfspaces; an infinite bound is absent),
             cap slack t_c >= 0
  objective  (gamma/2)(sum_i d_i w_i^2 + sum_j f_j y_j^2) - mu'^T w
             + kappa sum_i p_i + sum_ij (kappa + sigma_ij) s_ij, with
             mu' = eta mu + gamma Sigma w_b (the benchmark term of Eq. 1
             expanded; its constant does not move w*)
  equalities 1^T w = 1;  y - B^T w = 0;  R w - t = 0 (R: band rows by
             label, halfspace rows dense);
             w_i - p_i + sum_j s_ij = w0_i;  sum p + sum s + t_c = tau_eff

Because the tax slopes are non-decreasing, cheapest lots fill first, so the
lifted cost equals kappa|dw| + T((-dw)_+) exactly and w* is unchanged.
Excluded assets are fixed at 0 and removed; their trades are constants.

Each Newton step needs a solve with the normal matrix A H^-1 A^T, H the
diagonal Hessian plus barrier terms.  Two independent linear-algebra routes:

  "schur"  the link rows (one per asset) are decoupled from each other, so
           they are eliminated in closed form and a dense Schur complement on
           the few coupling rows (budget, k factor rows, bands, cap) is
           factored -- O(n (k+G)^2) per step;
  "sparse" the full augmented system [-H A^T; A 0] assembled with
           scipy.sparse and factored by SuperLU (small/medium n only).

Test infrastructure only.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .problem import AccountProblem, box, rows_bounds, linear_term


@dataclass
class Lifted:
    """Index bookkeeping and data of the lifted QP."""
    E: np.ndarray          # eligible asset indices (n_e)
    k: int
    G: int
    lift: bool
    has_cap: bool
    # per sale variable: owning eligible position (0..n_e-1) and lot number
    s_owner: np.ndarray
    s_lot: np.ndarray
    # variable layout
    nw: int
    ny: int
    np_: int
    ns: int
    nt: int
    nc: int
    q: np.ndarray          # diagonal Hessian
    c: np.ndarray          # linear cost
    lo: np.ndarray         # lower bounds (-inf allowed)
    hi: np.ndarray         # upper bounds (+inf allowed)
    b: np.ndarray          # equality right-hand side
    BE: np.ndarray         # B rows of eligible assets (n_e, k)
    gE: np.ndarray         # group labels of eligible assets (or empty)
    Gl: int                # band rows (by label); rows Gl..G-1 are halfspaces
    hE: np.ndarray         # halfspace rows on the eligible assets (G - Gl, n_e)
    const: float           # objective constant from excluded assets

    @property
    def nvar(self):
        return self.nw + self.ny + self.np_ + self.ns + self.nt + self.nc

    @property
    def n_link(self):
        return self.nw if self.lift else 0

    @property
    def n_coup(self):
        return 1 + self.k + self.G + (1 if self.has_cap else 0)

    # slices
    def sw(self):
        return slice(0, self.nw)

    def sy(self):
        o = self.nw
        return slice(o, o + self.ny)

    def sp(self):
        o = self.nw + self.ny
        return slice(o, o + self.np_)

    def ss(self):
        o = self.nw + self.ny + self.np_
        return slice(o, o + self.ns)

    def st(self):
        o = self.nw + self.ny + self.np_ + self.ns
        return slice(o, o + self.nt)

    def sc(self):
        o = self.nw + self.ny + self.np_ + self.ns + self.nt
        return slice(o, o + self.nc)


def _phi_excluded(P: AccountProblem, i):
    """Constant trade cost of an excluded asset forced from w0_i to 0."""
    dw = -float(P.w0[i])
    cost = P.kappa * abs(dw)
    hit = np.nonzero(P.tax_asset == i)[0]
    if len(hit) and dw < 0:
        j = int(hit[0])
        s = -dw
        edges = [0.0, *P.tax_brk[j], np.inf]
        for L in range(4):
            if s > edges[L]:
                cost += P.tax_slope[j][L] * (min(s, edges[L + 1]) - edges[L])
    return cost


def lift(P: AccountProblem) -> Lifted:
    E = np.nonzero(P.eligible)[0]
    X = np.nonzero(~P.eligible)[0]
    n_e = len(E)
    k = P.k
    Gl = P.n_groups
    H = 0 if P.half is None else P.half.shape[0]
    G = Gl + H
    has_tax = len(P.tax_asset) > 0
    has_cap = bool(np.isfinite(P.tau))
    lift_ = bool(P.kappa > 0 or has_tax or has_cap)

    const = float(sum(_phi_excluded(P, i) for i in X))
    tau_eff = P.tau - float(np.abs(P.w0[X]).sum()) if has_cap else np.inf

    # tax lots of eligible assets
    pos = -np.ones(P.n, dtype=np.int64)
    pos[E] = np.arange(n_e)
    lot_of = {}
    for j, i in enumerate(P.tax_asset):
        if pos[i] >= 0:
            lot_of[int(pos[i])] = j
    s_owner, s_lot, s_len, s_cost = [], [], [], []
    if lift_:
        for e in range(n_e):
            if e in lot_of:
                j = lot_of[e]
                brk = P.tax_brk[j]
                lens = [brk[0], brk[1] - brk[0], brk[2] - brk[1], np.inf]
                for L in range(4):
                    s_owner.append(e)
                    s_lot.append(L)
                    s_len.append(lens[L])
                    s_cost.append(P.kappa + P.tax_slope[j][L])
            else:
                s_owner.append(e)
                s_lot.append(0)
                s_len.append(np.inf)
                s_cost.append(P.kappa)
    s_owner = np.asarray(s_owner, dtype=np.int64)
    s_lot = np.asarray(s_lot, dtype=np.int64)
    s_len = np.asarray(s_len, dtype=np.float64)
    s_cost = np.asarray(s_cost, dtype=np.float64)

    nw, ny = n_e, k
    np_ = n_e if lift_ else 0
    ns = len(s_owner)
    nt = G
    nc = 1 if (lift_ and has_cap) else 0

    lbv, ubv = box(P)
    row_lo, row_hi = rows_bounds(P)
    q = np.concatenate([P.gamma * P.d[E], P.gamma * P.f,
                        np.zeros(np_ + ns + nt + nc)])
    c = np.concatenate([-linear_term(P)[E], np.zeros(ny),
                        np.full(np_, P.kappa), s_cost, np.zeros(nt + nc)])
    lo = np.concatenate([lbv[E], np.full(ny, -np.inf),
                         np.zeros(np_ + ns), row_lo,
                         np.zeros(nc)])
    hi = np.concatenate([ubv[E], np.full(ny, np.inf),
                         np.full(np_, np.inf), s_len, row_hi,
                         np.full(nc, np.inf)])
    # equality rows: [budget, factor (k), band (G), cap] then link rows
    b_coup = np.concatenate([[1.0], np.zeros(k), np.zeros(G),
                             [tau_eff] if nc else np.zeros(0)])
    b_link = P.w0[E] if lift_ else np.zeros(0)
    b = np.concatenate([b_coup, b_link])
    return Lifted(E=E, k=k, G=G, lift=lift_, has_cap=bool(nc),
                  s_owner=s_owner, s_lot=s_lot,
                  nw=nw, ny=ny, np_=np_, ns=ns, nt=nt, nc=nc,
                  q=q, c=c, lo=lo, hi=hi, b=b,
                  BE=P.B[E], gE=(P.group[E] if Gl else np.zeros(0, np.int64)),
                  Gl=Gl, hE=(np.asarray(P.half, dtype=np.float64)[:, E] if H
                             else np.zeros((0, n_e))),
                  const=const)


# --------------------------------------------------------------------------
# the equality operator A (coupling rows first, then link rows)
# --------------------------------------------------------------------------
def A_mul(L: Lifted, x):
    w, y = x[L.sw()], x[L.sy()]
    out = [np.array([w.sum()]), y - L.BE.T @ w]
    if L.G:
        rw = np.concatenate([np.bincount(L.gE, weights=w, minlength=L.Gl), L.hE @ w])
        out.append(rw - x[L.st()])
    if L.nc:
        out.append(np.array([x[L.sp()].sum() + x[L.ss()].sum() + x[L.sc()][0]]))
    if L.lift:
        link = w - x[L.sp()] + np.bincount(L.s_owner, weights=x[L.ss()],
                                           minlength=L.nw)
        out.append(link)
    return np.concatenate(out)


def AT_mul(L: Lifted, lam):
    """A^T lam."""
    k, G = L.k, L.G
    o = 0
    lb_ = lam[o]; o += 1
    lf = lam[o:o + k]; o += k
    lg = lam[o:o + G]; o += G
    lc = 0.0
    if L.nc:
        lc = lam[o]; o += 1
    ll = lam[o:o + L.n_link]
    gw = np.full(L.nw, lb_) - L.BE @ lf
    if G:
        gw = gw + L.hE.T @ lg[L.Gl:]
        if L.Gl:
            gw = gw + lg[:L.Gl][L.gE]
    if L.lift:
        gw = gw + ll
    gy = lf.copy()
    gp = (np.full(L.np_, lc) - ll) if L.lift else np.zeros(0)
    gs = (lc + ll[L.s_owner]) if L.lift else np.zeros(0)
    gt = -lg
    gc = np.array([lc]) if L.nc else np.zeros(0)
    return np.concatenate([gw, gy, gp, gs, gt, gc])


def A_sparse(L: Lifted):
    """The same operator assembled as a scipy.sparse matrix (route "sparse")."""
    rows, cols, vals = [], [], []
    nv = L.nvar
    r = 0
    W = np.arange(L.nw)
    # budget
    rows += [np.zeros(L.nw, np.int64)]; cols += [W]; vals += [np.ones(L.nw)]
    r = 1
    # factor rows: y_j - sum_i B_ij w_i
    for j in range(L.k):
        rows += [np.full(L.nw, r, np.int64), np.array([r])]
        cols += [W, np.array([L.sy().start + j])]
        vals += [-L.BE[:, j], np.array([1.0])]
        r += 1
    for g in range(L.G):
        if g < L.Gl:
            members = W[L.gE == g]
            coef = np.ones(len(members))
        else:
            members = W
            coef = L.hE[g - L.Gl]
        rows += [np.full(len(members), r, np.int64), np.array([r])]
        cols += [members, np.array([L.st().start + g])]
        vals += [coef, np.array([-1.0])]
        r += 1
    if L.nc:
        P_ = np.arange(L.sp().start, L.sp().stop)
        S_ = np.arange(L.ss().start, L.ss().stop)
        idx = np.concatenate([P_, S_, [L.sc().start]])
        rows += [np.full(len(idx), r, np.int64)]
        cols += [idx]
        vals += [np.ones(len(idx))]
        r += 1
    if L.lift:
        link_r = r + W
        rows += [link_r, link_r, r + L.s_owner]
        cols += [W, L.sp().start + W, L.ss().start + np.arange(L.ns)]
        vals += [np.ones(L.nw), -np.ones(L.nw), np.ones(L.ns)]
        r += L.nw
    A = sp.csr_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(r, nv))
    return A


# --------------------------------------------------------------------------
# normal-equation solves
# --------------------------------------------------------------------------
class SchurSolver:
    """Solves (A H^-1 A^T) u = r by eliminating the link rows."""

    def __init__(self, L: Lifted, h):
        self.L = L
        hi = 1.0 / h
        hw = hi[L.sw()]
        self.hi = hi
        k, G = L.k, L.G
        m = L.n_coup
        # coupling rows restricted to w: C_w (m x n_e)
        Cw = np.zeros((m, L.nw))
        Cw[0] = 1.0
        Cw[1:1 + k] = -L.BE.T
        if L.Gl:
            Cw[1 + k + L.gE, np.arange(L.nw)] = 1.0
        if G > L.Gl:
            Cw[1 + k + L.Gl:1 + k + G] = L.hE
        NCC = (Cw * hw) @ Cw.T
        NCC[np.arange(1, 1 + k), np.arange(1, 1 + k)] += hi[L.sy()]
        if G:
            NCC[np.arange(1 + k, 1 + k + G), np.arange(1 + k, 1 + k + G)] += \
                hi[L.st()]
        if L.nc:
            NCC[m - 1, m - 1] += hi[L.sp()].sum() + hi[L.ss()].sum() + \
                hi[L.sc()][0]
        if L.lift:
            hs_sum = np.bincount(L.s_owner, weights=hi[L.ss()], minlength=L.nw)
            NLL = hw + hi[L.sp()] + hs_sum
            NLC = (Cw * hw).T.copy()                 # (n_e x m)
            if L.nc:
                NLC[:, m - 1] += -hi[L.sp()] + hs_sum
            S = NCC - (NLC / NLL[:, None]).T @ NLC
            self.NLL, self.NLC = NLL, NLC
        else:
            S = NCC
        # S is positive definite in exact arithmetic; late in the iteration
        # the elimination of the lifted rows can cancel it to indefinite in
        # float64, and an LU factorization then takes over
        try:
            self.cho, self.lu = sla.cho_factor(S, lower=True), None
        except np.linalg.LinAlgError:
            self.cho, self.lu = None, sla.lu_factor(S)

    def _solve_s(self, rc):
        if self.cho is not None:
            return sla.cho_solve(self.cho, rc)
        return sla.lu_solve(self.lu, rc)

    def solve(self, r):
        L = self.L
        m = L.n_coup
        rc, rl = r[:m], r[m:]
        if L.lift:
            rc = rc - self.NLC.T @ (rl / self.NLL)
            uc = self._solve_s(rc)
            ul = (rl - self.NLC @ uc) / self.NLL
            return np.concatenate([uc, ul])
        return self._solve_s(rc)


def _newton_sparse(L: Lifted, Asp, h, xi, rp):
    """Solve [H -A^T; A 0][dx; dlam] = [xi; -rp] directly (route "sparse")."""
    n = L.nvar
    m = Asp.shape[0]
    K = sp.bmat([[sp.diags(h), -Asp.T], [Asp, None]], format="csc")
    rhs = np.concatenate([xi, -rp])
    sol = spla.splu(K).solve(rhs)
    return sol[:n], sol[n:n + m]


# --------------------------------------------------------------------------
# Mehrotra predictor-corrector
# --------------------------------------------------------------------------
@dataclass
class IPMResult:
    w: np.ndarray          # full-length weights
    nu: float
    lam_band: np.ndarray
    lam_cap: float
    iters: int
    converged: bool
    pres: float
    dres: float
    gap: float


def _initial_point(L: Lifted, P: AccountProblem):
    x = np.zeros(L.nvar)
    n_e = L.nw
    lbE, ubE = L.lo[L.sw()], L.hi[L.sw()]
    span = ubE - lbE
    theta = (1.0 - lbE.sum()) / max(span.sum(), 1e-300)
    theta = min(max(theta, 0.05), 0.95)
    w = lbE + theta * span
    x[L.sw()] = w
    x[L.sy()] = L.BE.T @ w
    if L.lift:
        # trades that satisfy the link rows w - p + sum_j s_j = w0 exactly:
        # bounded lots start mid-lot, the buy and the last (unbounded) sale
        # variable absorb the rest with a margin delta
        delta = 0.1 * span
        dw = w - P.w0[L.E]
        sv = np.zeros(L.ns)
        fin = np.isfinite(L.hi[L.ss()])
        sv[fin] = 0.5 * L.hi[L.ss()][fin]
        s_bnd = np.bincount(L.s_owner, weights=sv, minlength=n_e)
        p = np.maximum(dw + s_bnd, 0.0) + delta
        last = np.zeros(n_e, dtype=np.int64)
        last[L.s_owner[~fin]] = np.nonzero(~fin)[0]
        sv[last] = p - s_bnd - dw
        x[L.sp()] = p
        x[L.ss()] = sv
    if L.G:
        # the rows' values at the starting weights, moved inside their
        # bounds below (a one-sided row has no midpoint)
        x[L.st()] = np.concatenate([np.bincount(L.gE, weights=w, minlength=L.Gl),
                                    L.hE @ w])
        tlo, thi = L.lo[L.st()], L.hi[L.st()]
        both_t = np.isfinite(tlo) & np.isfinite(thi)
        rw = x[L.st()]
        # one-sided rows: a tenth of the values' scale inside the finite bound
        # (a start 1e-12 inside it is badly centred)
        with np.errstate(invalid="ignore"):
            margin = 0.1 * np.maximum(np.maximum(np.abs(np.where(np.isfinite(thi), thi, tlo)),
                                                 np.abs(rw)), 1e-8)
        t = np.where(np.isfinite(thi) & ~both_t, np.minimum(rw, thi - margin), rw)
        t = np.where(np.isfinite(tlo) & ~both_t, np.maximum(t, tlo + margin), t)
        x[L.st()] = np.where(both_t, 0.5 * (tlo + thi), t)
    if L.nc:
        x[L.sc()] = max(0.5 * L.b[L.n_coup - 1], 1e-3)
    # strictly inside bounds
    lo, hi = L.lo, L.hi
    both = np.isfinite(lo) & np.isfinite(hi)
    marg = np.where(both, 0.05 * (hi - lo), 0.0)
    x = np.where(np.isfinite(lo), np.maximum(x, lo + np.maximum(marg, 1e-12)),
                 x)
    x = np.where(np.isfinite(hi), np.minimum(x, hi - np.maximum(marg, 1e-12)),
                 x)
    return x


def solve_ipm(P: AccountProblem, route: str = "schur", tol: float = 1e-12,
              max_iter: int = 200) -> IPMResult:
    L = lift(P)
    if L.nw == 0:
        raise ValueError("no eligible asset")
    Asp = A_sparse(L) if route == "sparse" else None
    amul = (lambda x: Asp @ x) if Asp is not None else (lambda x: A_mul(L, x))
    atmul = (lambda v: Asp.T @ v) if Asp is not None else \
        (lambda v: AT_mul(L, v))

    x = _initial_point(L, P)
    m = L.n_coup + L.n_link
    lam = np.zeros(m)
    fl = np.isfinite(L.lo)
    fu = np.isfinite(L.hi)
    # centred start: every complementarity pair begins at the same value
    # mu0, chosen from the cost scale times a typical slack
    sl0 = np.where(fl, x - L.lo, np.inf)
    su0 = np.where(fu, L.hi - x, np.inf)
    slack_typ = float(np.median(np.minimum(sl0, su0)[fl | fu]))
    mu0 = max(float(np.max(np.abs(L.c))), 1e-3) * slack_typ
    zl = np.where(fl, mu0 / np.where(fl, x - L.lo, 1.0), 0.0)
    zu = np.where(fu, mu0 / np.where(fu, L.hi - x, 1.0), 0.0)
    nb = int(fl.sum() + fu.sum())
    bnorm = 1.0 + float(np.max(np.abs(L.b)))
    cnorm = 1.0 + float(np.max(np.abs(L.c)))

    def resid(x, lam, zl, zu):
        rd = L.q * x + L.c - atmul(lam) - zl + zu
        rp = amul(x) - L.b
        return rd, rp

    converged = False
    it = 0
    best = np.inf
    stall = 0
    pres = dres = gap = np.inf
    # bound slacks are iterates of their own (recomputing hi - x from x loses
    # every digit once x is within a few ulps of a bound)
    sl = np.where(fl, x - L.lo, 1.0)
    su = np.where(fu, L.hi - x, 1.0)
    for it in range(1, max_iter + 1):
        rd, rp = resid(x, lam, zl, zu)
        mu_c = (float((sl * zl)[fl].sum()) + float((su * zu)[fu].sum())) / \
            max(nb, 1)
        pres = float(np.max(np.abs(rp))) / bnorm
        dres = float(np.max(np.abs(rd))) / cnorm
        # worst single complementarity pair, not the average: one pair left at
        # 1e-12 can keep a coordinate micro-units away from its kink
        gap = max(float(np.max((sl * zl)[fl], initial=0.0)),
                  float(np.max((su * zu)[fu], initial=0.0)))
        if pres < tol and dres < tol and gap < tol * 1e-4:
            converged = True
            break
        merit = max(pres, dres, mu_c * 1e4)
        if merit < 0.9 * best:
            best, stall = merit, 0
        else:
            stall += 1
            if stall >= 10:          # no progress: round-off floor reached
                break
        h = L.q + np.where(fl, zl / sl, 0.0) + np.where(fu, zu / su, 0.0)
        h = np.maximum(h, 1e-300)
        solver = SchurSolver(L, h) if Asp is None else None

        def newton(cl, cu, sigma_mu):
            xi = -rd + np.where(fl, (sigma_mu - sl * zl - cl) / sl, 0.0) \
                - np.where(fu, (sigma_mu - su * zu - cu) / su, 0.0)
            if solver is not None:
                rhs = -rp - amul(xi / h)
                dlam = solver.solve(rhs)
                # iterative refinement against the unformed normal matrix
                # A H^-1 A^T (its formed Schur complement loses digits to
                # cancellation when h spans many orders of magnitude)
                for _ in range(2):
                    dlam = dlam + solver.solve(rhs - amul(atmul(dlam) / h))
                dx = (xi + atmul(dlam)) / h
            else:
                dx, dlam = _newton_sparse(L, Asp, h, xi, rp)
            dzl = np.where(fl, (sigma_mu - sl * zl - cl - zl * dx) / sl, 0.0)
            dzu = np.where(fu, (sigma_mu - su * zu - cu + zu * dx) / su, 0.0)
            return dx, dlam, dzl, dzu

        def max_step(dx, dzl, dzu):
            a = 1.0
            for v, dv, msk in ((sl, dx, fl), (su, -dx, fu), (zl, dzl, fl),
                               (zu, dzu, fu)):
                neg = msk & (dv < 0)
                if neg.any():
                    a = min(a, float(np.min(-v[neg] / dv[neg])))
            return a

        zero = np.zeros(L.nvar)
        dx_a, dl_a, dzl_a, dzu_a = newton(zero, zero, 0.0)
        a_aff = max_step(dx_a, dzl_a, dzu_a)
        sl_a = sl + a_aff * dx_a
        su_a = su - a_aff * dx_a
        zl_a = zl + a_aff * dzl_a
        zu_a = zu + a_aff * dzu_a
        mu_aff = (float((sl_a * zl_a)[fl].sum()) +
                  float((su_a * zu_a)[fu].sum())) / max(nb, 1)
        sigma = (mu_aff / max(mu_c, 1e-300)) ** 3
        cl = np.where(fl, dx_a * dzl_a, 0.0)
        cu = np.where(fu, (-dx_a) * dzu_a, 0.0)
        dx, dl, dzl, dzu = newton(cl, cu, sigma * mu_c)
        a = min(1.0, 0.995 * max_step(dx, dzl, dzu))
        x = x + a * dx
        sl = np.where(fl, sl + a * dx, 1.0)
        su = np.where(fu, su - a * dx, 1.0)
        lam = lam + a * dl
        zl = zl + a * dzl
        zu = zu + a * dzu
        # keep strictly interior against round-off
        zl = np.where(fl, np.maximum(zl, 1e-300), 0.0)
        zu = np.where(fu, np.maximum(zu, 1e-300), 0.0)

    w = np.zeros(P.n)
    w[L.E] = x[L.sw()]
    # multipliers: lam holds the equality duals of A x = b with the
    # convention grad = A^T lam + zl - zu.  Budget row: grad_w has +nu, and
    # the build's convention writes stationarity as grad - nu + A^T lam_band.
    nu = float(lam[0])
    lam_band = -lam[1 + L.k:1 + L.k + L.G] if L.G else np.zeros(0)
    lam_cap = float(-lam[L.n_coup - 1]) if L.nc else 0.0
    return IPMResult(w=w, nu=nu, lam_band=lam_band, lam_cap=lam_cap, iters=it,
                     converged=converged, pres=pres, dres=dres, gap=gap)
