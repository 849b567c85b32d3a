"""GPU parity of the two layouts of the turnover-cap multiplier search and
of the certification schedule.

The register-resident layout serves books with n <= 16384 and at most 2048
held names per account (the first 1024 held rows keep their tax records in
registers, the rest re-read theirs at every evaluation); every other book
takes the streaming layout.  The headline-shaped tests exercise the first
1024 held rows only, so these books cross each boundary."""
import numpy as np
import pytest

from workloads import make_config
from _gpu_helpers import run_gpu, check_account
from test_gpu_full_sizes import _all_certified_by_cpu_checker

pytestmark = pytest.mark.gpu


def _held_counts(book):
    return np.diff(np.asarray(book.tax_ptr))


def test_resident_layout_past_1024_held_rows():
    uni, book = make_config("c3", 3, N=6000, M=4, k=16, held=(1500, 1800))
    H = _held_counts(book)
    assert H.max() > 1024 and H.max() <= 2048 and np.all(np.isfinite(book.tau))
    print("case resident, held", H.tolist(), flush=True)
    host, st = run_gpu(uni, book, rho=5.0)
    for a in range(book.m):
        check_account(uni, book, a, host)


def test_streaming_layout_many_held_names():
    uni, book = make_config("c3", 4, N=5000, M=3, k=16, held=(2100, 2300))
    H = _held_counts(book)
    assert H.max() > 2048 and np.all(np.isfinite(book.tau))
    print("case streaming (held), held", H.tolist(), flush=True)
    host, st = run_gpu(uni, book, rho=5.0)
    for a in range(book.m):
        check_account(uni, book, a, host)


def test_streaming_layout_wide_universe():
    uni, book = make_config("c3", 5, N=20000, M=3, k=16)
    assert uni.n > 16384 and np.all(np.isfinite(book.tau))
    print("case streaming (n = 20000)", flush=True)
    host, st = run_gpu(uni, book, rho=8.0, alpha=1.8)
    assert int(np.sum(host["status"] == 0)) == book.m
    _all_certified_by_cpu_checker(uni, book, host)
    check_account(uni, book, 0, host)


def test_first_check_delays_certification_only():
    uni, book = make_config("c3", 1, N=1300, M=9, k=16)
    print("case first_check 150, check_every 50", flush=True)
    host, st = run_gpu(uni, book, rho=5.0, check_every=50, first_check=150)
    assert int(host["iters"].min()) >= 150
    assert np.all(host["iters"] % 50 == 0)
    for a in range(book.m):
        check_account(uni, book, a, host)
