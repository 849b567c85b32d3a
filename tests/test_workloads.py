"""The seeded synthetic books: determinism, float32 exactness, and the
feasibility facts the problem class relies on (Slater's condition for the
budget-box program, Sec. "Benchmark Problem Class"; a strictly feasible
turnover cap)."""
import numpy as np
import pytest

from workloads import make_config, subset_accounts
from workloads.books import to_f32_exact


@pytest.mark.parametrize("name,over", [
    ("c1", {}), ("c2", dict(N=500, M=4)), ("c3", dict(N=2000, M=5)),
    ("c4", dict(N=500, M=3)), ("c5", dict(N=5000, M=2, held=(300, 300))),
])
def test_deterministic_and_f32(name, over):
    u1, b1 = make_config(name, 3, **over)
    u2, b2 = make_config(name, 3, **over)
    for x, y in [(u1.B, u2.B), (u1.d, u2.d), (b1.mu, b2.mu), (b1.w0, b2.w0),
                 (b1.tax_brk, b2.tax_brk), (b1.tau, b2.tau)]:
        assert np.array_equal(x, y)
    for x in [u1.B, u1.f, u1.d, b1.mu, b1.w0, b1.tax_brk, b1.tax_slope,
              b1.ub, b1.gamma, b1.kappa]:
        assert np.array_equal(x, to_f32_exact(x))
    u3, _ = make_config(name, 4, **over)
    assert not np.array_equal(u1.B, u3.B)


def test_account_data_independent_of_book_size():
    _, small = make_config("c3", 0, N=1000, M=3)
    _, big = make_config("c3", 0, N=1000, M=7)
    assert np.array_equal(small.mu, big.mu[:3])
    assert np.array_equal(small.w0, big.w0[:3])


def test_c3_shape_and_feasibility():
    uni, book = make_config("c3", 0, N=10000, M=20)
    assert uni.B.shape == (10000, 80)
    frac = book.eligible.mean(axis=1)
    assert frac.min() >= 0.3 - 1e-9 and frac.max() <= 1.0
    for a in range(book.m):
        held = np.count_nonzero(book.w0[a])
        assert 100 <= held <= 400
        assert np.all(book.w0[a] <= book.ub[a] + 1e-9)
        # Slater: sum of eligible upper bounds > 1
        assert book.eligible[a].sum() * book.ub[a] > 1.0
        # strictly feasible cap: tau >= tau_min + 0.1 - rounding
        u = np.where(book.eligible[a], book.ub[a], 0.0)
        tau_min = 2 * np.maximum(book.w0[a] - u, 0).sum()
        assert book.tau[a] >= tau_min + 0.1 - 1e-6
        ta, tb, ts = book.tax_of(a)
        assert np.all(np.diff(ta) > 0)
        assert np.all(np.diff(tb, axis=1) > 0) and np.all(tb[:, 0] > 0)
        assert np.all(tb[:, 2] < book.w0[a, ta])
        assert np.all(np.diff(ts, axis=1) >= 0) and np.all(ts >= 0)


def test_subset_accounts_roundtrip():
    _, book = make_config("c3", 1, N=800, M=6)
    sub = subset_accounts(book, [4, 1])
    assert np.array_equal(sub.mu[0], book.mu[4])
    for j, a in enumerate([4, 1]):
        for x, y in zip(sub.tax_of(j), book.tax_of(a)):
            assert np.array_equal(x, y)
