"""GPU: per-account audit records and queue accounting of a batched solve."""
import numpy as np
import pytest

from workloads import make_config

pytestmark = pytest.mark.gpu


def test_audit_records_are_consistent_and_deterministic():
    import torch
    from paper_2606_23367_amd.solver import Solver, to_device
    from paper_2606_23367_amd.audit import audit_records, queue_summary
    uni, book = make_config("c3", 21, N=1300, M=9, k=16)
    P = to_device(uni, book)
    s = Solver(0)
    print("case audit c3 N=1300 M=9", flush=True)
    runs = []
    for _ in range(2):
        out = s.solve(P, rho=5.0)
        torch.cuda.synchronize()
        runs.append((audit_records(P, out, s), s.pass_times(), s.stats()["total_ms"]))
    (r1, passes, total), (r2, _, _) = runs
    assert [r["input_sha256"] for r in r1] == [r["input_sha256"] for r in r2]
    assert [r["output_sha256"] for r in r1] == [r["output_sha256"] for r in r2]
    assert len(set(r["input_sha256"] for r in r1)) == book.m
    iters = [it for it, _ in passes]
    ms = [t for _, t in passes]
    assert iters == sorted(iters) and ms == sorted(ms) and ms[-1] <= total
    for r in r1:
        assert r["status"] == "certified"
        assert r["iterations"] in iters
        assert r["completed_ms"] == ms[iters.index(r["iterations"])]
    q = queue_summary(r1, budget_ms=500.0)
    assert q["completed"] == book.m and q["miss_rate"] == 0.0
    assert q["t_queue_ms"] == max(r["completed_ms"] for r in r1)
