"""Autotuner of the ADMM schedule and of the iteration passes' layout.

Schedule: penalty rho, over-relaxation alpha, the certification interval
check_every, the delay of the first certification pass (first_check = a
multiple of check_every) and the active-set refinement rounds of each pass
(polish_rounds).  Layout, tried for the winning schedule: the rows of one
iteration-pass workgroup (tile_rows, 0 = sized from the occupancy) and the
contraction precision (bf16-split or float32 MFMA).

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
                    check_every=(50, 100), first_mult=(1, 2, 3), polish_rounds=(8, 16, 24))
# layouts tried for the winning schedule: tile_rows (in 128-row chunks; 0 =
# from the occupancy) x precision (1 = bf16-split, 0 = float32 MFMA)
DEFAULT_LAYOUTS = dict(tile_rows=(0, 1, 2, 4), precision=(1, 0))

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
             finalists: int, layouts: Optional[dict] = None) -> str:
    """Cache key: the book's shape plus everything that changes the search
    (grid, layouts, sample size, how many more books confirm the finalists)."""
    g = ";".join(f"{k}={','.join(str(v) for v in grid[k])}" for k in sorted(grid))
    lay = "" if not layouts else "|L" + ";".join(
        f"{k}={','.join(str(v) for v in layouts[k])}" for k in sorted(layouts))
    return f"{shape_key(P, precision)}|s{sample}|b{n_second}|f{finalists}|{g}{lay}"


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
             finalists: int = 3, use_cache: bool = True,
             layouts: Optional[dict] = DEFAULT_LAYOUTS) -> dict:
    """Settings dict {rho, alpha, check_every, first_check, polish_rounds (when
    the grid has it), precision, tile_rows (when layouts are searched)} for
    books shaped like P, from timed solves of its first ``sample`` accounts
    (and of the first ``sample`` accounts of each book in ``second`` for the
    best ``finalists``).  ``layouts`` (None: keep ``precision`` and the
    occupancy-sized tiles) are then timed with the winning schedule on the
    same books.  ``use_cache=False`` always searches (and then refreshes the
    cache)."""
    grid = grid or DEFAULT_GRID
    others = [] if second is None else (
        [second] if isinstance(second, DeviceProblem) else list(second))
    key = tune_key(P, precision, grid, sample, len(others), finalists, layouts)
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
    for rho, alpha, ce, fm, pr in itertools.product(grid["rho"], grid["alpha"],
                                                    grid["check_every"],
                                                    grid.get("first_mult", (1,)),
                                                    grid.get("polish_rounds", (None,))):
        cfg = dict(rho=float(rho), alpha=float(alpha), check_every=int(ce),
                   first_check=int(fm) * int(ce), precision=precision)
        if pr is not None:
            cfg["polish_rounds"] = int(pr)
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
    if layouts:
        books = [Q] + [subset(B, range(min(sample, B.m))) for B in others]
        lay = []
        for tr, prec in itertools.product(layouts.get("tile_rows", (0,)),
                                          layouts.get("precision", (precision,))):
            cfg = dict(best[1], tile_rows=int(tr), precision=int(prec))
            ok_t, dt_t = 0, 0.0
            for B in books:
                s.solve(B, **cfg)                          # warm-up of this layout
                # the layouts differ by about a percent: the better of two
                # timings per book keeps one noisy run from deciding
                (ok, dt), (_, dt2) = _timed(s, B, cfg), _timed(s, B, cfg)
                ok_t += ok
                dt_t += min(dt, dt2)
            if verbose:
                print(f"autotune layout {cfg}: {ok_t} certified, {dt_t * 1e3:.1f} ms", flush=True)
            lay.append(((-ok_t, dt_t), cfg))
        lay.sort(key=lambda r: r[0])
        best = lay[0]
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
