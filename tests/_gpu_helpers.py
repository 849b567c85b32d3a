"""Shared helpers of the GPU tests: run the HIP solver through the C-ABI and
compare with the float64 oracle on the same seeded inputs."""
import numpy as np

import oracle
from oracle.problem import account, n_rows
from oracle.kkt import residuals

# Acceptance of the headline target (1e-6 relative objective, 1e-6 primal
# and dual residual, measured by the oracle's own checker on the GPU output)
TOL_OBJ = 1e-6
TOL_PRIM = 1e-6
TOL_DUAL = 1e-6
TOL_COMP = 1e-6


def weight_error_bound(P, obj_gap):
    """Largest ||w - w*||_2 a feasible w with f(w) - f(w*) <= obj_gap can
    have: f is strongly convex with modulus gamma * min(d) (Sigma - diag(d)
    is PSD), so f(w) - f(w*) >= (gamma min d / 2) ||w - w*||^2."""
    m = P.gamma * float(np.min(P.d))
    return float(np.sqrt(2.0 * max(obj_gap, 0.0) / m))


def run_gpu(uni, book, solver=None, **settings):
    import torch
    from paper_2606_23367_amd.solver import Solver, to_device
    P = to_device(uni, book)
    s = solver or Solver(0)
    out = s.solve(P, **settings)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in out.items()}
    return host, s.stats()


def check_account(uni, book, a, host):
    P = account(uni, book, a)
    orc = oracle.solve_account(P)
    # the oracle's own answer is certified far below the GPU tolerances
    assert max(orc["res"]["r_prim"], orc["res"]["r_dual"],
               orc["res"]["r_comp"]) <= 1e-11, orc["res"]
    w = host["w"][a]
    lam_band = host["lam_band"][a] if n_rows(P) else None
    r = residuals(P, w, host["nu"][a], lam_band, host["lam_cap"][a])
    relobj = abs(r["obj"] - orc["obj"]) / max(abs(orc["obj"]), 1e-300)
    info = dict(a=a, status=int(host["status"][a]), r_prim=r["r_prim"],
                r_dual=r["r_dual"], r_comp=r["r_comp"], relobj=relobj,
                werr=float(np.max(np.abs(w - orc["w"]))))
    assert host["status"][a] == 0, info
    assert r["r_prim"] <= TOL_PRIM, info
    assert r["r_dual"] <= TOL_DUAL, info
    assert r["r_comp"] <= TOL_COMP, info
    assert relobj <= TOL_OBJ, info
    # the weights: within what the objective gap allows (plus the residual
    # primal infeasibility and round-off of the two objective evaluations)
    gap = r["obj"] - orc["obj"] + 1e-13 * max(abs(orc["obj"]), 1.0)
    werr2 = float(np.linalg.norm(w - orc["w"]))
    info["werr2"] = werr2
    info["werr2_bound"] = weight_error_bound(P, gap) + 10 * r["r_prim"]
    assert werr2 <= info["werr2_bound"], info
    # the GPU's own float64 diagnostics agree with the oracle's checker
    check_reported_diagnostics(host, a, r, info)
    return info


def check_reported_diagnostics(host, a, r, info=None):
    """The residuals and objective the GPU reports for account a (its own
    float64 certification) equal what the CPU checker computes from the
    returned weights and multipliers."""
    info = info if info is not None else dict(a=a)
    info.update(gpu_r_prim=float(host["r_prim"][a]), gpu_r_dual=float(host["r_dual"][a]),
                gpu_r_comp=float(host["r_comp"][a]))
    assert abs(host["r_prim"][a] - r["r_prim"]) <= 1e-9, info
    assert abs(host["r_dual"][a] - r["r_dual"]) <= 1e-9, info
    assert abs(host["r_comp"][a] - r["r_comp"]) <= 1e-9, info
    assert abs(host["obj"][a] - r["obj"]) <= 1e-12 * max(1.0, abs(r["obj"])), info
