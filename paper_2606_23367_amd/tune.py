"""Autotuner of the ADMM schedule: penalty rho, over-relaxation alpha, the
certification interval check_every and the delay of the first
certification pass (first_check = a multiple of check_every).

The right penalty depends on the scale of the book (box width, return
spread, risk aversion) and the interval trades polish attempts against
iterations (an early pass over a full batch costs a float64 polish of every
account and certifies few of them), so all are picked by timing solves of a
sample of accounts over a small grid.  The winner certifies the most sampled accounts, then
takes the least time.  The wall time of a batch is set by its slowest
accounts, which makes single timings of nearby settings noisy; with more
books of the same shape the best few settings are timed again on them and
ranked by all books together.  Results are cached per book shape
(in memory, and in a JSON file when a path is given); tune on accounts
that are not the ones being timed.
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Optional, Sequence, Union

import torch

from .solver import DeviceProblem, Solver, subset

DEFAULT_GRID = dict(rho=(1.0, 3.0, 6.0, 8.0, 10.0, 14.0, 30.0), alpha=(1.6, 1.8),
                    check_every=(50, 100), first_mult=(1, 2))

_CACHE: dict = {}


def shape_key(P: DeviceProblem, precision: int) -> str:
    """Book features the schedule depends on (not the account data)."""
    has_tax = P.tax_ptr is not None and int(P.tax_ptr[-1].item()) > 0
    has_cap = bool(torch.isfinite(P.tau).any().item())
    ub = float(P.ub.max().item())
    lb = float(P.lb.min().item())
    gam = float(P.gamma.max().item())
    kap = float(P.kappa.max().item())
    extra = "".join(tag for tag, x in (("_half", P.half_lo), ("_abox", P.lb_asset),
                                       ("_wb", P.wb), ("_eta", P.eta)) if x is not None)
    return (f"n{P.n}_k{P.k}_g{P.G}h{P.H}{extra}_tax{int(has_tax)}_cap{int(has_cap)}"
            f"_elig{int(P.eligible is not None)}_lb{lb:.3g}_ub{ub:.3g}_gam{gam:.3g}"
            f"_kap{kap:.3g}_p{precision}")


def tune_key(P: DeviceProblem, precision: int, grid: dict, sample: int, n_second: int,
             finalists: int) -> str:
    """Cache key: the book's shape plus everything that changes the search
    (grid, sample size, how many more books confirm the finalists)."""
    g = ";".join(f"{k}={','.join(str(v) for v in grid[k])}" for k in sorted(grid))
    return f"{shape_key(P, precision)}|s{sample}|b{n_second}|f{finalists}|{g}"


def clear_cache() -> None:
    """Forget the in-memory picks (the JSON file, if any, is kept)."""
    _CACHE.clear()


def _timed(s: Solver, Q: DeviceProblem, cfg: dict):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = s.solve(Q, **cfg)
    torch.cuda.synchronize()
    return int((out["status"] == 0).sum().item()), time.perf_counter() - t0


def autotune(P: DeviceProblem, solver: Optional[Solver] = None, sample: int = 64,
             grid: Optional[dict] = None, precision: int = 1,
             cache_path: Optional[str] = None, verbose: bool = False,
             second: Union[DeviceProblem, Sequence[DeviceProblem], None] = None,
             finalists: int = 3, use_cache: bool = True) -> dict:
    """Settings dict {rho, alpha, check_every, first_check, precision} for
    books shaped like P, from timed solves of its first ``sample`` accounts (and of the
    first ``sample`` accounts of each book in ``second`` for the best ``finalists``).
    ``use_cache=False`` always searches (and then refreshes the cache)."""
    grid = grid or DEFAULT_GRID
    others = [] if second is None else (
        [second] if isinstance(second, DeviceProblem) else list(second))
    key = tune_key(P, precision, grid, sample, len(others), finalists)
    if use_cache and key in _CACHE:
        return dict(_CACHE[key])
    if use_cache and cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            disk = json.load(fh)
        if key in disk:
            _CACHE[key] = disk[key]
            return dict(disk[key])
    s = solver or Solver(P.mu.device.index or 0)
    Q = subset(P, range(min(sample, P.m)))
    s.solve(Q, precision=precision)                       # warm-up: workspace, code
    ranked = []
    for rho, alpha, ce, fm in itertools.product(grid["rho"], grid["alpha"], grid["check_every"],
                                                grid.get("first_mult", (1,))):
        cfg = dict(rho=float(rho), alpha=float(alpha), check_every=int(ce),
                   first_check=int(fm) * int(ce), precision=precision)
        ok, dt = _timed(s, Q, cfg)
        if verbose:
            print(f"autotune {cfg}: {ok}/{Q.m} certified, {dt * 1e3:.1f} ms", flush=True)
        ranked.append(((-ok, dt), cfg))
    ranked.sort(key=lambda r: r[0])
    best = ranked[0]
    if others and finalists > 1:
        fin = [[score[0], score[1], cfg] for (score, cfg) in ranked[:finalists]]
        for B in others:
            Q2 = subset(B, range(min(sample, B.m)))
            s.solve(Q2, precision=precision)              # warm-up
            for f in fin:
                ok2, dt2 = _timed(s, Q2, f[2])
                if verbose:
                    print(f"autotune other book {f[2]}: {ok2}/{Q2.m} certified, "
                          f"{dt2 * 1e3:.1f} ms", flush=True)
                f[0] -= ok2
                f[1] += dt2
        fin.sort(key=lambda f: (f[0], f[1]))
        best = ((fin[0][0], fin[0][1]), fin[0][2])
    _CACHE[key] = best[1]
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                disk = json.load(fh)
        disk[key] = best[1]
        with open(cache_path, "w") as fh:
            json.dump(disk, fh, indent=1, sort_keys=True)
    return dict(best[1])
