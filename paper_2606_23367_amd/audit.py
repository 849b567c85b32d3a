"""Per-account audit records and queue accounting of one batched solve.

The paper's production queue reports, per account, an input and an output
digest, the status and the elapsed time, and for the queue the completion
count, percentiles of the completion time and the share of accounts that
miss a per-account budget (Sec. "Production Queue", Sec. "Status Vocabulary
and Objective Agreement").  In a batched solve every account shares one
call; an account certified after i ADMM iterations is complete at the end of
the certification pass run after i iterations (``Solver.pass_times``), and
an account that never certified at the end of the call.
"""
from __future__ import annotations

import hashlib
from typing import Optional

import numpy as np

from ._lib import STATUS_NAMES, SOLVED, FEASIBLE_UNCERTIFIED


def _host(t):
    return None if t is None else t.detach().cpu().numpy()


def audit_records(P, out: dict, solver) -> list:
    """One record per account of the last ``solver.solve(P)`` whose outputs
    are ``out``: input_sha256 over the account's data (returns, holdings,
    box, eligibility, scalars, bands, tax lots, and the halfspace bounds,
    per-asset bounds, benchmark and return scale when given), output_sha256 over its
    float64 weights, status, iterations and completed_ms."""
    passes = solver.pass_times()
    total_ms = solver.stats()["total_ms"]
    done_at = {it: ms for it, ms in passes}
    mu, w0, lb, ub = _host(P.mu), _host(P.w0), _host(P.lb), _host(P.ub)
    elig, gam, kap, tau = _host(P.eligible), _host(P.gamma), _host(P.kappa), _host(P.tau)
    blo, bhi = _host(P.band_lo), _host(P.band_hi)
    tptr, tas, tbr, tsl = _host(P.tax_ptr), _host(P.tax_asset), _host(P.tax_brk), _host(P.tax_slope)
    w, status, iters = _host(out["w"]), _host(out["status"]), _host(out["iters"])
    extra = [x for x in (_host(getattr(P, name, None)) for name in
                         ("half_lo", "half_hi", "lb_asset", "ub_asset", "wb", "eta"))
             if x is not None]
    recs = []
    for a in range(P.m):
        h = hashlib.sha256()
        for arr in (mu[a], w0[a], lb[a:a + 1], ub[a:a + 1], gam[a:a + 1], kap[a:a + 1],
                    tau[a:a + 1]):
            h.update(np.ascontiguousarray(arr).tobytes())
        if elig is not None:
            h.update(np.ascontiguousarray(elig[a]).tobytes())
        if blo is not None and P.G:
            h.update(np.ascontiguousarray(blo[a]).tobytes())
            h.update(np.ascontiguousarray(bhi[a]).tobytes())
        if tptr is not None:
            s, e = int(tptr[a]), int(tptr[a + 1])
            for arr in (tas[s:e], tbr[s:e], tsl[s:e]):
                h.update(np.ascontiguousarray(arr).tobytes())
        for arr in extra:                       # the rest of Eq. 1, when given
            h.update(np.ascontiguousarray(arr[a]).tobytes())
        st = int(status[a])
        it = int(iters[a])
        recs.append({
            "account": a,
            "input_sha256": h.hexdigest(),
            "output_sha256": hashlib.sha256(np.ascontiguousarray(w[a]).tobytes()).hexdigest(),
            "status": STATUS_NAMES.get(st, str(st)),
            "status_code": st,
            "iterations": it,
            "completed_ms": done_at.get(it, total_ms) if st == SOLVED else total_ms,
        })
    return recs


def queue_summary(records: list, budget_ms: Optional[float] = None) -> dict:
    """Queue figures of a batch: T_queue (the last completion), completion
    count (returns that pass the external gates: certified or feasible
    uncertified), p50 / p99 completion time, status counts and, with a
    per-account budget, the share of accounts completed late or not at
    all."""
    t = np.array([r["completed_ms"] for r in records], dtype=float)
    codes = [r["status_code"] for r in records]
    completed = sum(c in (SOLVED, FEASIBLE_UNCERTIFIED) for c in codes)
    counts = {}
    for r in records:
        counts[r["status"]] = counts.get(r["status"], 0) + 1
    out = {"accounts": len(records), "completed": completed,
           "t_queue_ms": float(t.max()) if len(t) else 0.0,
           "p50_ms": float(np.percentile(t, 50)) if len(t) else 0.0,
           "p99_ms": float(np.percentile(t, 99)) if len(t) else 0.0,
           "status_counts": counts}
    if budget_ms is not None:
        late = sum((c not in (SOLVED, FEASIBLE_UNCERTIFIED)) or (ti > budget_ms)
                   for c, ti in zip(codes, t))
        out["budget_ms"] = budget_ms
        out["miss_rate"] = late / max(len(records), 1)
    return out
