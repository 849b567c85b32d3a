"""CPU checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-side entry points behave without a GPU."""
import ctypes
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fqp.h")).read()
    return sorted(set(re.findall(r"FQP_API\s+[\w\s\*]*?\b(fqp_\w+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("fqp_create", "fqp_solve_batch", "fqp_destroy",
                 "fqp_default_settings", "fqp_get_stats"):
        assert must in names


def test_library_loads_and_exports_every_symbol():
    from paper_2606_23367_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) <= set(_lib.EXPORTS)


def test_host_entry_points_without_gpu():
    from paper_2606_23367_amd import _lib
    lib = _lib.load()
    s = _lib.Settings()
    lib.fqp_default_settings(ctypes.byref(s))
    assert s.eps_prim == 1e-6 and s.eps_dual == 1e-6 and s.max_iter > 0
    assert lib.fqp_error_string(-1) == b"invalid argument"
    assert lib.fqp_status_string(0) == b"certified"
    st = _lib.Stats()
    assert lib.fqp_get_stats(None, ctypes.byref(st)) == -1
    lib.fqp_destroy(None)


def test_struct_layouts_match_header():
    """sizeof of every ABI struct, compiled from the header with gcc."""
    import subprocess
    import tempfile
    from paper_2606_23367_amd import _lib
    src = ('#include <stdio.h>\n#include "fqp.h"\nint main(){printf("%zu %zu '
           '%zu %zu %zu %zu\\n", sizeof(fqp_universe), sizeof(fqp_book), '
           'sizeof(fqp_settings), sizeof(fqp_result), sizeof(fqp_stats), '
           'sizeof(int));}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o",
                        exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True,
                             check=True).stdout.split()
    sizes = [ctypes.sizeof(t) for t in (_lib.Universe, _lib.Book,
                                        _lib.Settings, _lib.Result,
                                        _lib.Stats)]
    assert [int(x) for x in out[:5]] == sizes


def test_eligibility_packing():
    import numpy as np
    from paper_2606_23367_amd.solver import pack_eligibility
    rng = np.random.default_rng(0)
    e = rng.random((3, 70)) < 0.5
    w = pack_eligibility(e)
    assert w.shape == (3, 3)
    for a in range(3):
        for i in range(70):
            assert bool((int(w[a, i // 32]) >> (i % 32)) & 1) == e[a, i]


def test_device_subset_matches_host_subset():
    """solver.subset on a (CPU-resident) device book equals laying out the
    host subset directly: same rows, re-based tax lots."""
    import torch
    from workloads import make_config, subset_accounts
    from paper_2606_23367_amd.solver import to_device, subset
    uni, book = make_config("c3", 1, N=300, M=6, k=4)
    P = to_device(uni, book, "cpu")
    idx = [4, 1, 5]
    A = subset(P, idx)
    B = to_device(uni, subset_accounts(book, idx), "cpu")
    for name in ("mu", "w0", "lb", "ub", "gamma", "kappa", "tau", "eligible",
                 "tax_ptr", "tax_asset", "tax_brk", "tax_slope"):
        a, b = getattr(A, name), getattr(B, name)
        assert (a is None) == (b is None), name
        if a is not None:
            assert torch.equal(a, b), name
    assert A.m == 3


def test_queue_summary_counts_and_percentiles():
    from paper_2606_23367_amd.audit import queue_summary
    from paper_2606_23367_amd._lib import SOLVED, FEASIBLE_UNCERTIFIED, MAX_ITER, STATUS_NAMES
    codes = [SOLVED] * 7 + [FEASIBLE_UNCERTIFIED, MAX_ITER, SOLVED]
    times = [10.0, 10.0, 20.0, 20.0, 20.0, 30.0, 30.0, 40.0, 40.0, 600.0]
    recs = [{"status_code": c, "status": STATUS_NAMES[c], "completed_ms": t}
            for c, t in zip(codes, times)]
    q = queue_summary(recs, budget_ms=500.0)
    assert q["accounts"] == 10 and q["completed"] == 9
    assert q["t_queue_ms"] == 600.0
    assert q["p50_ms"] == float(np.percentile(times, 50))
    assert q["p99_ms"] == float(np.percentile(times, 99))
    assert q["status_counts"][STATUS_NAMES[SOLVED]] == 8
    # the iteration-cap account and the one past the budget
    assert q["miss_rate"] == 0.2
