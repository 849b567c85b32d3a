"""Float64 CPU oracle for the batched factor-model rebalancing QP.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never calls it, and it shares no code with the GPU library.

It computes the unique minimiser of the build's instance of the paper's
Eq. 1 (Sec. "Benchmark Problem Class") for each account: a Mehrotra
interior-point method on a lifted QP (``oracle.ipm``) followed by an exact
crossover (``oracle.crossover``), and the external diagnostics of Sec.
"External Diagnostics" (``oracle.kkt``).

Pins (tests marked ``not gpu``): the closed-form budget-only solution, brute
force active-set enumeration for N <= 8, a separable (B = 0) case solved by
nested bisection, two independent linear-algebra routes, and the KKT
residuals themselves.
"""
from __future__ import annotations

import numpy as np

from .problem import AccountProblem, account, objective, objective_scale  # noqa
from .kkt import residuals  # noqa: F401
from .ipm import solve_ipm
from .crossover import crossover


def _score(out):
    r = out["res"]
    return max(r["r_prim"], r["r_dual"], r["r_comp"])


def solve_account(P: AccountProblem, route: str = "schur", tol=1e-12,
                  max_iter=200, certify=1e-11):
    """Oracle solution of one account: dict with w, nu, lam_band, lam_cap,
    res (external diagnostics), method, route, ipm_iters.

    When the requested linear-algebra route does not reach a point the
    crossover certifies to ``certify`` (the dense Schur complement can lose
    definiteness to cancellation late in the iteration), the other route
    is run and the better answer kept."""
    best = None
    routes = [route] + [r for r in ("schur", "sparse") if r != route]
    for rt in routes:
        r = solve_ipm(P, route=rt, tol=tol, max_iter=max_iter)
        out = crossover(P, r.w, r.nu, r.lam_band, r.lam_cap)
        out["ipm_iters"] = r.iters
        out["ipm_converged"] = r.converged
        out["route"] = rt
        out["obj"] = out["res"]["obj"]
        if best is None or _score(out) < _score(best):
            best = out
        if r.converged and _score(best) <= certify:
            break
    return best


def solve_book(uni, book, accounts=None, **kw):
    """Solve accounts of a book one by one (list of dicts)."""
    idx = range(book.m) if accounts is None else accounts
    return [solve_account(account(uni, book, int(a)), **kw) for a in idx]
