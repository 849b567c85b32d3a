"""Throughput of the batched rebalancing solver on one MI355X.

One step = one fqp_solve_batch call on the headline book (500 accounts over
an N = 10,000 universe, k = 80 factors, exclusion masks leaving 30-100 % of
names eligible, 4-lot piecewise-linear tax on 100-400 held names, turnover
cap): packing and validation, factor-space setup, ADMM iterations, float64
polish and certification of every account.  Inputs are resident in HBM when
the timed region starts; the timed steps run the library's captured-graph
path.  value = accounts certified to 1e-6 KKT residuals per second.

The roofline object describes the iteration pass that takes the most time
per solve (PROX, CONTRACT or PROJECT): algorithmic bytes per launch / average
launch duration, both from one more (untimed) solve whose pass launches are
timed with events that each dispatch stamps (hipExtLaunchKernelGGL) on the
library's stream.

plain_fp32 is the same book solved one account per call with float32
contractions (the unbatched form), on a bounded sample of accounts.

cpu_baseline times the float64 oracle on a bounded sample of the same book
on the host cores, and states the GPU's error against it per account.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "c3"
# the ADMM schedule (rho, alpha, check_every, first_check) is picked by the
# autotuner on the books of other seeds of the same shape (grid on the
# first, the finalists confirmed on three more); bf16-split contractions
# (the library default)
TUNE_SEED, TUNE_SEEDS2, TUNE_SAMPLE = 1, (2, 3, 4), 500
SETTINGS = dict(precision=1)


def factor_width(uni):
    """Used columns of the factor block B~ = [B | band rows | halfspace rows | 1]."""
    return uni.k + uni.n_groups + getattr(uni, "n_half", 0) + 1


def algorithmic_bytes(uni, book, iters, precision, kind="project"):
    """Algorithmic bytes of one iteration pass over a solve, from the
    per-account iteration counts: (sum over account-iterations, per launch).

    PROX (the cap multiplier, then z, r and the two streams of the rest of
    the iteration): per account-iteration v and mu read, R' = r / Delta and
    w = v + alpha (R' - z) written (16 N), the eligibility bits (N / 8 when
    the book has exclusions) and one 28-byte tax record per held name; per
    launch d (4 N).

    CONTRACT (the contraction t = B~^T R'): per account-iteration R' read
    (4 N); per launch the used columns of B~ at 2 B per entry (the bf16
    width of the method's model) and d (4 N).

    PROJECT (back-projection and the write of the new ADMM state): per
    account-iteration w read and v written (8 N); per launch the used
    columns of B~ (bf16 hi and lo: 4 B per entry; float32: 4 B) and d
    (4 N)."""
    import numpy as np
    n = uni.n
    kw = factor_width(uni)
    if kind == "project":
        per_acc = np.full(book.m, 8.0 * n)
        per_launch = 4.0 * n * kw + 4.0 * n
    elif kind == "contract":
        per_acc = np.full(book.m, 4.0 * n)
        per_launch = 2.0 * n * kw + 4.0 * n
    else:
        held = np.count_nonzero(book.w0, axis=1)
        mask = 0.0 if book.eligible.all() else np.ceil(n / 8.0)
        per_acc = 16.0 * n + mask + 28.0 * held
        per_launch = 4.0 * n
    return float(np.sum(iters * per_acc)), float(per_launch)


TRAFFIC_NOTES = {
    "prox": os.path.join(ROOT, "profiles", "prox_pass_c3_500x10000_hbm_traffic.md"),
    "contract": os.path.join(ROOT, "profiles", "contract_pass_c3_500x10000_hbm_traffic.md"),
    "project": os.path.join(ROOT, "profiles", "project_pass_c3_500x10000_hbm_traffic.md"),
}
KERNEL_SOURCES = ["paper_2606_23367_amd/csrc/fqp_iter.hip", "paper_2606_23367_amd/csrc/fqp_common.h",
                  "paper_2606_23367_amd/csrc/fqp_kernels.h"]


def measured_traffic(kind):
    """HBM bytes per launch of the pass from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        txt = open(TRAFFIC_NOTES[kind]).read()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in txt.splitlines()
                if line.startswith(("traffic_bytes_per_launch: ", "kernel_sources_sha256: ")))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if vals.get("kernel_sources_sha256", "").strip() != h.hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"])


def timed_solves(solver, P, steps, settings, profile=0, prox=None):
    """Run `steps` solves; profile=0 is the library's captured-graph path,
    bits 0 / 1 / 2 time every PROJECT / CONTRACT / PROX launch with events
    (no graph; the PROX milliseconds are added to prox[0]).  Returns
    (seconds, certified, PROJECT ms, CONTRACT ms, launches, iters per
    solve)."""
    import torch
    out = None
    solved, proj_ms, con_ms, launches, iters = 0, 0.0, 0.0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = solver.solve(P, out=out, profile=profile, **settings)
        # the call returns with its statuses counted (stats.n_solved: the
        # accounts certified); the iteration counts are copied on the device
        # and read after the timed region, so no step waits on the host
        st = solver.stats()
        iters.append(out["iters"].clone())
        solved += int(st["n_solved"])
        proj_ms += st["iter_kernel_ms"]
        con_ms += st["contract_kernel_ms"]
        if prox is not None:
            prox[0] += st["prox_kernel_ms"]
        launches += st["iter_launches"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, solved, proj_ms, con_ms, launches, [x.cpu().numpy() for x in iters]


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Achievable HBM bandwidth: bytes read + written by a device-to-device
    copy of a 1 GiB buffer (larger than the 256 MB last-level cache), best
    of `reps`, timed with events on the current stream."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return 2.0 * nbytes / (best * 1e-3) / 1e9


MFMA_BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3            # dense float32 MFMA, MI355X


def mfma_report(uni, book, iters, project_ms, contract_ms, split=True):
    """Matrix-core rates of the two contraction passes over one profiled step:
    useful flops are the products with the k + G + H + 1 used columns of B~
    (2 N (k + G + H + 1) per account-iteration and pass); issued flops count
    the padded width kp and, on the bf16-split path, its three bf16 products
    per float32 product."""
    import numpy as np
    n, k, G = uni.n, uni.k, uni.n_groups + getattr(uni, "n_half", 0)
    kg1 = k + G + 1
    kp = ((kg1 + 31) // 32) * 32
    acc_iters = float(sum(np.sum(it) for it in iters))
    useful = 2.0 * n * kg1 * acc_iters              # per pass
    issued = useful * (3.0 if split else 1.0) * kp / kg1
    peak = MFMA_BF16_PEAK_TFLOPS if split else FP32_PEAK_TFLOPS
    out = {"instruction": "v_mfma_f32_32x32x16_bf16 (hi*hi + hi*lo + lo*hi)" if split
           else "v_mfma_f32_32x32x2_f32", "peak_tflops": peak}
    for name, ms in (("contract", contract_ms), ("project", project_ms)):
        if ms > 0:
            out[name] = {"useful_tflops": useful / (ms * 1e-3) / 1e12,
                         "issued_tflops": issued / (ms * 1e-3) / 1e12,
                         "issued_frac": issued / (ms * 1e-3) / 1e12 / peak}
    return out


def queue_lane(solver, P, settings, budget_ms=500.0):
    """Queue accounting of one more (untimed, graph-mode) solve of the timed
    book: completion count, T_queue, p50 / p99 per-account completion and
    the miss rate against a 0.5 s per-account budget (the paper's
    deadline-bounded scenario), from the per-account audit records."""
    import torch
    from paper_2606_23367_amd.audit import audit_records, queue_summary
    out = solver.solve(P, **settings)
    torch.cuda.synchronize()
    recs = audit_records(P, out, solver)
    q = queue_summary(recs, budget_ms=budget_ms)
    q["passes"] = [{"iterations": it, "ms": ms} for it, ms in solver.pass_times()]
    return q


def warm_lane(solver, uni, book, settings, sd=1e-4):
    """Repeated-rebalance lane: the same book with returns moved by
    N(0, sd^2) (about 1 % of their cross-sectional spread), solved cold with
    the timed schedule and warm from the previous day's ADMM state with a
    pass every 50 iterations; one solve each after the state-setting one."""
    import dataclasses
    import numpy as np
    import torch
    from workloads.books import to_f32_exact
    from paper_2606_23367_amd.solver import to_device
    rng = np.random.default_rng(2024)
    nxt = dataclasses.replace(book, mu=to_f32_exact(book.mu + rng.normal(0.0, sd, book.mu.shape)))
    P, P2 = to_device(uni, book), to_device(uni, nxt)
    warm_settings = dict(settings, check_every=50, first_check=50)
    res = {}
    for lane, cfg, first in (("cold", settings, P2), ("warm", dict(warm_settings, warm_start=1), P)):
        solver.solve(first, **(settings if lane == "warm" else cfg))   # yesterday / warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = solver.solve(P2, **cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        it = out["iters"].cpu().numpy()
        res[lane] = {"value": int((out["status"] == 0).sum().item()) / dt, "ms": dt * 1e3,
                     "account_iterations": int(it.sum()), "max_iterations": int(it.max())}
    res["unit"] = "accounts/s"
    res["returns_shift_sd"] = sd
    res["warm_schedule"] = {"check_every": 50, "first_check": 50}
    return res


# constraint-burden bundles at N = 2,000 (64 accounts, k = 40), cumulative:
# every bundle keeps the previous one's data and adds one rule family (B3:
# factor-exposure bounds, 5 halfspace rows on B^T w within 5e-3 of the
# equal-weight exposure; B5 puts tax lots on B4's holdings)
_B3 = dict(halfspaces=5, half_halfwidth=5e-3)
BURDEN = (
    ("B0 budget, long-only, box", dict(kappa=0.0, groups=0, band_halfwidth=None)),
    ("B1 + turnover penalty", dict(kappa=1e-3, groups=0, band_halfwidth=None)),
    ("B2 + sector bands", dict(kappa=1e-3)),
    ("B3 + factor-exposure bounds", dict(kappa=1e-3, **_B3)),
    ("B4 + account exclusions", dict(kappa=1e-3, elig=(0.3, 1.0), **_B3)),
    ("B5 + tax lots", dict(kappa=1e-3, elig=(0.3, 1.0), tax=True, **_B3)),
)
BURDEN_GRID = dict(rho=(0.3, 1.0, 3.0, 10.0), alpha=(1.8,), check_every=(25, 50),
                   polish_rounds=(4, 16))


def burden_lane(solver, steps=3):
    """Accounts/s of a 64 x 2,000 book as rule families accumulate (the
    paper's constraint-burden curve, synthetic): schedule tuned per bundle
    on its seed-1 book with the finalists confirmed on the seed-2 and seed-3
    books (schedules within a percent on one book can differ by a quarter on
    another), best of `steps` solves of the seed-0 book."""
    import torch
    from workloads import make_config
    from paper_2606_23367_amd.solver import to_device
    from paper_2606_23367_amd.tune import autotune
    rows = []
    for label, over in BURDEN:
        u1, b1 = make_config("c2", 1, **over)
        others = [to_device(*make_config("c2", sd, **over), "cuda:0") for sd in (2, 3)]
        cfg = autotune(to_device(u1, b1, "cuda:0"), solver=solver, sample=b1.m,
                       grid=BURDEN_GRID, second=others)
        uni, book = make_config("c2", 0, **over)
        P = to_device(uni, book, "cuda:0")
        solver.solve(P, **cfg)
        best, solved = None, 0
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = solver.solve(P, **cfg)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best:
                best, solved = dt, int((out["status"] == 0).sum().item())
        rows.append({"bundle": label, "ms_per_book": best * 1e3, "accounts_per_s": solved / best,
                     "certified": solved, "accounts": book.m, "rho": cfg["rho"],
                     "check_every": cfg["check_every"],
                     "polish_rounds": cfg.get("polish_rounds")})
    return rows


E7_GRID = dict(rho=(0.3, 1.0, 3.0, 10.0), alpha=(1.6, 1.8), check_every=(25, 50),
               first_mult=(1, 2), polish_rounds=(4, 8, 16))


def e7_lane(solver, steps=5):
    """Small-universe batch: 200 accounts over N = 481 names (k = 20, box
    [0, 0.03], L1 transition cost 5e-3, drifted holdings), the shape of the
    paper's 200-account real-data queue.  Schedule from the autotuner on the
    seed-1 book (finalists confirmed on seeds 2-4); the timed book is seed
    0; best of `steps` whole-book solves."""
    import numpy as np
    import torch
    from workloads import make_config
    from paper_2606_23367_amd.solver import to_device
    from paper_2606_23367_amd.tune import autotune
    u1, b1 = make_config("e7", 1)
    others = [to_device(*make_config("e7", sd), "cuda:0") for sd in (2, 3, 4)]
    cfg = autotune(to_device(u1, b1, "cuda:0"), solver=solver, sample=b1.m, grid=E7_GRID,
                   second=others)
    uni, book = make_config("e7", 0)
    P = to_device(uni, book, "cuda:0")
    solver.solve(P, **cfg)
    best, solved, its = None, 0, None
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = solver.solve(P, **cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if best is None or dt < best:
            best, solved, its = dt, int((out["status"] == 0).sum().item()), out["iters"].cpu().numpy()
    return {"value": solved / best, "unit": "accounts/s", "ms_per_book": best * 1e3,
            "accounts": book.m, "certified": solved, "assets": uni.n, "factors": uni.k,
            "settings": cfg, "iterations_p50_max": [float(np.median(its)), int(its.max())],
            "data": "synthetic stand-in for the paper's 481-name real universe"}


# E7-shaped variants: the L1 transition cost and the position cap of the
# paper's small-universe scenarios (5e-3 and 1e-2; caps of 3 % and 1.2 %)
E7_VARIANTS = ((5e-3, 0.03), (1e-2, 0.03), (5e-3, 0.012), (1e-2, 0.012))


def e7_variants_lane(solver, cfg, steps=3):
    """The e7 book (200 x 481) at every (transition cost, position cap) pair,
    with the schedule the autotuner picked for the base variant; best of
    `steps` solves each."""
    import torch
    from workloads import make_config
    from paper_2606_23367_amd.solver import to_device
    rows = []
    for kappa, cap in E7_VARIANTS:
        uni, book = make_config("e7", 0, kappa=kappa, ub=cap)
        P = to_device(uni, book, "cuda:0")
        solver.solve(P, **cfg)
        best, solved = None, 0
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = solver.solve(P, **cfg)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best:
                best, solved = dt, int((out["status"] == 0).sum().item())
        rows.append({"transition_cost": kappa, "position_cap": cap, "ms_per_book": best * 1e3,
                     "accounts_per_s": solved / best, "certified": solved, "accounts": book.m})
    return rows


def c5_lane(solver, steps=2):
    """Large universe: 8 accounts over N = 384,800 names, k = 100, 50 one-hot
    groups with bands, 2,000 held names with 4-lot tax (the factor block is
    151 columns wide, so the contractions run on float32 MFMA); best of
    `steps` solves after a warm-up."""
    import numpy as np
    import torch
    from workloads import make_config
    from paper_2606_23367_amd.solver import to_device
    uni, book = make_config("c5", 0)
    P = to_device(uni, book, "cuda:0")
    cfg = dict(rho=10.0)
    solver.solve(P, **cfg)
    best, solved, its = None, 0, None
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = solver.solve(P, **cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if best is None or dt < best:
            best, solved, its = dt, int((out["status"] == 0).sum().item()), out["iters"].cpu().numpy()
    del P
    return {"value": solved / best, "unit": "accounts/s", "ms_per_book": best * 1e3,
            "accounts": book.m, "certified": solved, "assets": uni.n, "factors": uni.k,
            "groups": uni.n_groups, "settings": cfg,
            "iterations_max": int(its.max()), "precision": "float32 MFMA contractions "
            "(factor block 151 columns)", "data": "synthetic"}


def c4_grad_lane(solver, steps=3):
    """Differentiation: 128 accounts over N = 5,000, k = 60, gamma = 1000 --
    a forward solve plus the KKT-adjoint backward for dL/dmu and dL/dB of
    L = sum_a c_a^T w_a; best of `steps` forward+backward passes."""
    import numpy as np
    import torch
    from workloads import make_config
    from paper_2606_23367_amd.solver import to_device
    uni, book = make_config("c4", 0)
    P = to_device(uni, book, "cuda:0")
    C = torch.as_tensor(np.random.default_rng(7).normal(size=(book.m, uni.n)), device="cuda:0")
    cfg = dict(rho=1.0)
    solver.solve(P, **cfg)
    solver.adjoint(C)
    best_f = best_b = None
    solved = 0
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = solver.solve(P, **cfg)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        solver.adjoint(C)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if best_f is None or (t2 - t0) < best_f + best_b:
            best_f, best_b = t1 - t0, t2 - t1
            solved = int((out["status"] == 0).sum().item())
    return {"value": solved / (best_f + best_b), "unit": "accounts/s (forward + backward)",
            "forward_ms": best_f * 1e3, "backward_ms": best_b * 1e3, "accounts": book.m,
            "certified": solved, "assets": uni.n, "factors": uni.k, "data": "synthetic"}


def plain_fp32(uni, book, n_sample):
    """The unbatched float32 form: one account per fqp_solve_batch call,
    float32 MFMA contractions, the first n_sample accounts."""
    from workloads import subset_accounts
    from paper_2606_23367_amd.solver import Solver, to_device
    settings = dict(SETTINGS, precision=0)    # same schedule, float32 contractions
    solver = Solver(0)
    probs = [to_device(uni, subset_accounts(book, [a]), "cuda:0") for a in range(n_sample)]
    timed_solves(solver, probs[0], 1, settings, profile=1)      # warm-up
    dt, solved, kms, launches, alg = 0.0, 0, 0.0, 0, 0.0
    for a, P in enumerate(probs):
        t, s, km, _, la, it = timed_solves(solver, P, 1, settings, profile=1)
        dt += t; solved += s; kms += km; launches += la
        per_acc, per_launch = algorithmic_bytes(uni, subset_accounts(book, [a]), it[0], 0)
        alg += per_acc + per_launch * la
    achieved = alg / (kms * 1e-3) / 1e9 if kms > 0 else None
    return dict(value=solved / dt, unit="accounts/s", sample=f"first {n_sample} accounts, "
                f"one per call, {solved} certified", precision="fp32 MFMA contractions",
                project_achieved_gbs=achieved,
                project_frac=(achieved / HBM_PEAK_GBS) if achieved else None,
                avg_launch_us=kms * 1e3 / max(launches, 1))


def cpu_baseline(uni, book, n_sample, gpu_out=None):
    """Oracle (float64 IPM + crossover) on the first n_sample accounts, one
    account per worker process, BLAS pinned to one thread per worker; the
    clock starts once every worker has built the book.  With the GPU's
    output of the same book, the GPU's error against the oracle on each
    sampled account: relative objective and the CPU checker's residuals of
    the GPU weights."""
    import multiprocessing as mp
    import numpy as np
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["OMP_NUM_THREADS"] = "1"
    cores = min(len(os.sched_getaffinity(0)), 16, n_sample)
    ctx = mp.get_context("spawn")
    ready = ctx.Barrier(cores + 1)          # every worker has built the book
    with ctx.Pool(cores, initializer=_pool_init, initargs=(ready,)) as pool:
        ready.wait(timeout=900)
        t0 = time.perf_counter()
        res = pool.map(_oracle_one, [(WORKLOAD, a) for a in range(n_sample)], chunksize=1)
        dt = time.perf_counter() - t0
    ok = sum(1 for r in res if r["certified"])
    line = dict(value=ok / dt, unit="accounts/s", cores=cores, kind="oracle",
                sample=f"first {n_sample} accounts of the 500-account book, "
                       f"{ok} certified, wall {dt:.1f} s after the workers built the book")
    if gpu_out is not None:
        from oracle.problem import account
        from oracle.kkt import residuals
        errs = []
        for a, r in enumerate(res):
            P = account(uni, book, a)
            lam_band = gpu_out["lam_band"][a] if uni.n_groups else None
            g = residuals(P, gpu_out["w"][a], gpu_out["nu"][a], lam_band, gpu_out["lam_cap"][a])
            errs.append((abs(g["obj"] - r["obj"]) / abs(r["obj"]), g["r_prim"], g["r_dual"],
                         g["r_comp"], float(np.max(np.abs(gpu_out["w"][a] - r["w"])))))
        e = np.asarray(errs)
        line["gpu_vs_oracle"] = {
            "accounts": len(errs),
            "rel_obj_max": float(e[:, 0].max()), "rel_obj_median": float(np.median(e[:, 0])),
            "r_prim_max": float(e[:, 1].max()), "r_dual_max": float(e[:, 2].max()),
            "r_comp_max": float(e[:, 3].max()), "weight_abs_err_max": float(e[:, 4].max()),
            "note": "GPU float64-polished weights of the timed solve against the float64 oracle "
                    "on the same accounts; residuals from the CPU checker",
        }
    return line


_POOL = {}


def _pool_init(ready):
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    from workloads import make_config
    _POOL["book"] = make_config(WORKLOAD, 0)
    ready.wait(timeout=900)


def _oracle_one(args):
    _, a = args
    import oracle
    from oracle.problem import account
    uni, book = _POOL["book"]
    out = oracle.solve_account(account(uni, book, a))
    r = out["res"]
    return {"certified": max(r["r_prim"], r["r_dual"], r["r_comp"]) <= 1e-6,
            "obj": out["obj"], "w": out["w"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=96)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=16,
                    help="accounts of the one-account-per-call float32 comparison")
    ap.add_argument("--no-lanes", action="store_true",
                    help="skip the extra reports (MFMA step, queue, warm, e7 and burden lanes): "
                         "the profiling runs")
    ap.add_argument("--schedule", default="", metavar="RHO,ALPHA,CHECK[,FIRST[,ROUNDS[,TILE]]]",
                    help="fixed ADMM schedule instead of the autotuner (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (the "
                         "reference kernel that scales HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: accounts are independent and "
              "multi-GPU sharding is not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}), flush=True)
        return
    from workloads import make_config
    from paper_2606_23367_amd.solver import Solver, to_device

    from paper_2606_23367_amd.tune import autotune
    solver = Solver(0)
    t_tune = time.perf_counter()
    if args.schedule:
        parts = args.schedule.split(",")
        tuned = dict(rho=float(parts[0]), alpha=float(parts[1]), check_every=int(parts[2]),
                     first_check=int(parts[3]) if len(parts) > 3 else 0)
        if len(parts) > 4:
            tuned["polish_rounds"] = int(parts[4])
        if len(parts) > 5:
            tuned["tile_rows"] = int(parts[5])
        settings_from = "fixed on the command line"
    else:
        tu_uni, tu_book = make_config(WORKLOAD, TUNE_SEED)
        others = [to_device(*make_config(WORKLOAD, sd), "cuda:0") for sd in TUNE_SEEDS2]
        tuned = autotune(to_device(tu_uni, tu_book, "cuda:0"), solver=solver,
                         sample=TUNE_SAMPLE, precision=SETTINGS["precision"], second=others)
        del others
        settings_from = None
    t_tune = time.perf_counter() - t_tune
    SETTINGS.update(tuned)
    uni, book = make_config(WORKLOAD, 0)
    P = to_device(uni, book, "cuda:0")
    cold_ms = None
    if args.warmup:
        t_cold = timed_solves(solver, P, 1, SETTINGS)[0]     # first call on this book
        cold_ms = t_cold * 1e3
        if args.warmup > 1:
            timed_solves(solver, P, args.warmup - 1, SETTINGS)
    # the timed steps: the library's captured-graph path
    dt, solved, _, _, launches, iters = timed_solves(solver, P, args.steps, SETTINGS)
    graph_reused = solver.stats()["graph_reused"]
    gpu_out = None
    if not args.no_cpu:
        last = solver.solve(P, **SETTINGS)
        torch.cuda.synchronize()
        gpu_out = {key: v.cpu().numpy() for key, v in last.items()}
    # one more (untimed) solve with every launch of both iteration passes
    # timed by events stamped at the kernels' own start and end
    pr_prox = [0.0]
    _, pr_solved, pr_proj_ms, pr_con_ms, pr_launches, pr_iters = timed_solves(
        solver, P, 1, SETTINGS, profile=7, prox=pr_prox)
    passes = {}
    for kind, ms in (("prox", pr_prox[0]), ("contract", pr_con_ms), ("project", pr_proj_ms)):
        per_acc, per_launch = algorithmic_bytes(uni, book, pr_iters[0], SETTINGS["precision"],
                                                kind)
        alg = per_acc + per_launch * pr_launches
        passes[kind] = {"ms_per_solve": ms, "launches": pr_launches,
                        "avg_launch_us": ms * 1e3 / max(pr_launches, 1),
                        "alg_bytes_per_launch": alg / max(pr_launches, 1),
                        "achieved_gbs": alg / (ms * 1e-3) / 1e9 if ms > 0 else None}
    dom = max(passes, key=lambda kd: passes[kd]["ms_per_solve"])
    it_all = np.concatenate(iters)
    # whole path against the per-account-iteration byte model of the method:
    # state z, u read + written, mu and w0 read (24 N), eligibility bits,
    # held records (28 B); B (4 B/entry), d and labels once per iteration
    held = np.count_nonzero(book.w0, axis=1)
    model = float(np.sum(np.concatenate([it * (24.0 * uni.n + np.ceil(uni.n / 8.0) + 28.0 * held)
                                         for it in iters])))
    model += float(np.sum([it.max() for it in iters])) * (4.0 * uni.n * uni.k + 4.0 * uni.n)

    value = solved / dt
    achieved = passes[dom]["achieved_gbs"]
    achievable = copy_bandwidth()
    split = SETTINGS["precision"] == 1
    kern = "iter_kernel_bf" if split else "iter_kernel"
    mm = "bf16-split MFMA" if split else "float32 MFMA"
    names = {"prox": "prox_kernel (exact turnover-cap multiplier, then z, r, R' = r / Delta "
                     "and w for every (account, asset))",
             "contract": f"{kern}<3, CONTRACT> ({mm} contraction B~^T R')",
             "project": f"{kern}<3, PROJECT> ({mm} back-projection B~p, new ADMM state)"}
    line = {
        "metric": "accounts solved/s to 1e-6 KKT residual (500 accts, N=10k), "
                  "% HBM roofline",
        "value": value,
        "unit": "accounts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"f32 ({mm}) + f64",
        "data": "synthetic",
        "config": {
            "workload": "500 accounts x N=10,000 assets, k=80 factors; "
                        "exclusion masks (30-100% eligible), 4-lot tax on "
                        f"100-400 held names, turnover cap; FP32 ADMM with {mm} "
                        "contractions + FP64 polish and certification",
            "settings": SETTINGS,
            "settings_from": settings_from or (
                f"autotune on {TUNE_SAMPLE} accounts of the seed-{TUNE_SEED} book of the "
                f"same shape, finalists confirmed on the books of seeds "
                f"{', '.join(str(x) for x in TUNE_SEEDS2)} ({t_tune:.1f} s, untimed)"),
            "accounts": book.m, "assets": uni.n, "factors": uni.k,
            "certified_per_step": solved / args.steps,
            "iter_launches_per_step": launches / args.steps,
            "iterations_p50_p90_p99_max": [float(np.percentile(it_all, q)) for q in (50, 90, 99)]
                                          + [int(it_all.max())],
            "cold_call_ms": cold_ms,
            "timed_path": "captured hipGraph per block of iterations (graph_reused="
                          f"{graph_reused} on the last timed call)",
        },
        "whole_path": {
            "model_bytes_per_step": model / args.steps,
            "effective_gbs": model / dt / 1e9,
            "frac": model / dt / 1e9 / HBM_PEAK_GBS,
            "note": "24N + N/8 + 28 H bytes per account-iteration plus B, d per iteration, "
                    "over the whole step (setup, iterations, polish, certification)",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": measured_traffic(dom),
            "kernel": names[dom],
            "alg_bytes_per_launch": passes[dom]["alg_bytes_per_launch"],
            "avg_launch_us": passes[dom]["avg_launch_us"],
            "achievable_gbs": achievable,
            "frac_of_achievable": (achieved / achievable) if (achieved and achievable) else None,
            "note": "the pass with the largest time per solve, from one more solve whose "
                    "launches are timed by events the dispatches stamp",
        },
        "passes": passes,
        "mfma": mfma_report(uni, book, pr_iters, pr_proj_ms, pr_con_ms, split),
    }
    if not args.no_lanes:
        line["queue"] = queue_lane(solver, P, SETTINGS)
        line["warm_lane"] = warm_lane(solver, uni, book, SETTINGS)
        e7 = e7_lane(solver)
        line["e7_lane"] = e7
        line["e7_variants"] = e7_variants_lane(solver, e7["settings"])
        line["burden_lane"] = burden_lane(solver)
        line["c4_grad_lane"] = c4_grad_lane(solver)
        del P
        torch.cuda.empty_cache()
        line["c5_lane"] = c5_lane(solver)
    if args.plain_sample > 0:
        line["plain_fp32"] = plain_fp32(uni, book, args.plain_sample)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(uni, book, args.cpu_sample, gpu_out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
