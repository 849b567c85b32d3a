"""GPU parity: the HIP path (through the C-ABI) against the float64 oracle
on the same seeded books, at sizes that span several row tiles and account
tiles with ragged tails, and sampled at the full headline size."""
import numpy as np
import pytest

from workloads import make_config, subset_accounts
from _gpu_helpers import run_gpu, check_account

pytestmark = pytest.mark.gpu

SMALL = [
    ("c1", {}, dict(rho=0.05)),
    ("c1", dict(N=37, ub=0.13), dict(rho=0.05)),             # N < 64, ragged
    ("c2", dict(N=700, M=40, k=10), dict(rho=1.0)),          # 2 account tiles
    ("c3", dict(N=1300, M=9, k=16), dict(rho=5.0)),          # masks, tax, cap
    ("c3", dict(N=37, M=3, k=4, ub=0.2, held=(3, 8)), dict(rho=5.0)),   # tiny, binding caps
    ("c4", dict(N=900, M=5, k=12), dict(rho=1.0)),           # gamma = 1000
    ("c4", dict(N=900, M=5, k=12, gamma=1.0), dict(rho=1.0)),
    ("c5", dict(N=6000, M=2, k=20, held=(300, 300)), dict(rho=10.0)),
    # factor blocks wider than the bf16-split passes take (k + G + 1 > 96):
    # float32 contraction passes and the factor-space setup in global
    # scratch; 151 columns (k = 100, G = 50) and 169 columns (k = 128, G = 40)
    ("c5", dict(N=20000, M=3, k=100, held=(300, 300)), dict(rho=10.0)),
    ("c5", dict(N=4100, M=2, k=128, groups=40, held=(200, 200)), dict(rho=10.0)),
    # every rule family at once: L1 turnover, sector bands, exclusions, taxed lots
    ("c2", dict(N=700, M=8, k=10, elig=(0.3, 1.0), held=(50, 120), tax=True), dict(rho=1.0)),
    # the polish passes' 512-row blocks: exactly two blocks, a last block of
    # one row, a single full block
    ("c3", dict(N=1024, M=6, k=8, held=(20, 60)), dict(rho=5.0)),
    ("c3", dict(N=513, M=5, k=8, held=(20, 60)), dict(rho=5.0)),
    ("c3", dict(N=512, M=5, k=8, held=(20, 60)), dict(rho=5.0)),
]


@pytest.mark.parametrize("name,over,settings", SMALL)
@pytest.mark.parametrize("seed", [0, 1])
def test_small_books_match_oracle(name, over, settings, seed):
    uni, book = make_config(name, seed, **over)
    print(f"case {name} {over} seed {seed}", flush=True)
    host, st = run_gpu(uni, book, **settings)
    for a in range(book.m):
        check_account(uni, book, a, host)


def test_large_free_set_takes_the_factor_space_polish():
    """A wide long-short box: every asset is free at the optimum, more than
    the 64 rows the row-space solve of the polish takes, so the polish
    solves in factor space."""
    uni, book = make_config("c1", 3, N=400, M=4)
    book.lb[:] = -1.0
    book.ub[:] = 1.0
    print("case c1 N=400 long-short", flush=True)
    host, st = run_gpu(uni, book, rho=0.05)
    for a in range(book.m):
        check_account(uni, book, a, host)
    assert all(np.sum(np.abs(host["w"][a]) > 1e-9) > 64 for a in range(book.m))


def test_headline_book_sampled():
    """500 accounts x N=10,000, k=80: every account certified; a sample
    checked against the oracle one by one."""
    uni, book = make_config("c3", 0)
    host, st = run_gpu(uni, book, rho=5.0)
    print("stats", st, flush=True)
    assert int(np.sum(host["status"] == 0)) == book.m
    for a in (0, 137, 499):
        check_account(uni, book, a, host)


def test_headline_book_at_the_bench_schedule():
    """The headline book at the schedule bench.py times (rho 8, alpha 1.8,
    a pass every 100 iterations from iteration 200): all 500 certified, the
    GPU's reported diagnostics equal the CPU checker's on every account,
    three accounts against the oracle."""
    from oracle.problem import account
    from oracle.kkt import residuals
    from _gpu_helpers import check_reported_diagnostics
    uni, book = make_config("c3", 0)
    host, st = run_gpu(uni, book, rho=8.0, alpha=1.8, check_every=100, first_check=200)
    print("stats", st, flush=True)
    assert int(np.sum(host["status"] == 0)) == book.m
    for a in range(book.m):
        P = account(uni, book, a)
        r = residuals(P, host["w"][a], host["nu"][a], None, host["lam_cap"][a])
        assert max(r["r_prim"], r["r_dual"], r["r_comp"]) <= 1e-6, (a, r)
        check_reported_diagnostics(host, a, r)
    for a in (0, 250, 499):
        check_account(uni, book, a, host)


def test_positive_lower_bound_with_masks_and_binding_cap():
    """lb > 0 (a minimum holding for eligible names) with exclusion masks,
    taxed holdings and a turnover cap close to its least feasible value, at
    N = 3,000 (not a multiple of the 1,024-row slices of the cap search):
    excluded names and the padding rows must stay at 0 in every pass."""
    from workloads.books import to_f32_exact
    uni, book = make_config("c3", 8, N=3000, M=6, k=12)
    lb = float(to_f32_exact(2e-5))
    book.lb[:] = lb
    for a in range(book.m):
        el = book.eligible[a]
        c = np.clip(book.w0[a], np.where(el, lb, 0.0), np.where(el, book.ub[a], 0.0))
        tmin = np.abs(book.w0[a] - c).sum() + abs(1.0 - c.sum())
        book.tau[a] = float(to_f32_exact(tmin + 0.05))
    host, st = run_gpu(uni, book, rho=5.0)
    for a in range(book.m):
        check_account(uni, book, a, host)
    assert np.all(host["w"][~book.eligible] == 0.0)
    assert np.any(host["lam_cap"] > 0.0)


def test_invalid_accounts_do_not_poison_batch():
    uni, book = make_config("c3", 3, N=900, M=7, k=8)
    book.lb[1], book.ub[1] = 0.02, 0.01                      # lb > ub
    book.eligible[2, :] = False
    book.eligible[2, :50] = True                             # 50 * 0.01 < 1
    book.tau[3] = 0.0 if book.tau[3] > 0.5 else book.tau[3] * 0.1  # tau < tau_min
    book.mu[4, 5] = np.nan
    s, e = book.tax_ptr[5], book.tax_ptr[6]
    if e > s:
        book.tax_slope[s, 0] = 0.01                          # decreasing slopes
        book.tax_slope[s, 1] = 0.001
    host, _ = run_gpu(uni, book, rho=5.0)
    assert host["status"][1] == 5           # invalid input
    assert host["status"][2] == 4           # primal infeasible (Slater)
    assert host["status"][3] == 4           # cap below the least turnover
    assert host["status"][4] == 6           # non-finite input
    if e > s:
        assert host["status"][5] == 5
    for a in (0, 6):
        check_account(uni, book, a, host)


def test_book_with_no_valid_account():
    # every account rejected at set-up: the iteration passes see an empty
    # active list, no iteration is counted and every output keeps its status
    from paper_2606_23367_amd.solver import Solver
    uni, book = make_config("c3", 3, N=700, M=4, k=8)
    for a in range(book.m):
        book.lb[a], book.ub[a] = 0.02, 0.01                  # lb > ub
    s = Solver(0)
    host, st = run_gpu(uni, book, solver=s, rho=5.0)
    assert np.all(host["status"] == 5)
    assert np.all(host["iters"] == 0)
    assert st["iterations"] == 0 and st["n_solved"] == 0
    assert np.all(host["w"] == 0.0) and np.all(np.isnan(host["obj"]))
    # the same handle then solves a valid book of the same shape
    uni2, book2 = make_config("c3", 3, N=700, M=4, k=8)
    host2, _ = run_gpu(uni2, book2, solver=s, rho=5.0)
    for a in range(book2.m):
        check_account(uni2, book2, a, host2)


def test_call_counters_match_the_outputs():
    # the certified count and the account-iterations the library reports
    # (reduced on the device into pinned host memory) equal what the
    # outputs show, over two calls of different books on one handle (the
    # second with invalid accounts and a smaller batch)
    from paper_2606_23367_amd.solver import Solver
    s = Solver(0)
    for seed, M in ((7, 9), (8, 5)):
        uni, book = make_config("c3", seed, N=1100, M=M, k=8)
        if seed == 8:
            book.lb[1], book.ub[1] = 0.02, 0.01              # invalid account
        host, st = run_gpu(uni, book, solver=s, rho=5.0)
        assert st["n_solved"] == int(np.sum(host["status"] == 0))
        assert st["account_iters"] == float(np.sum(host["iters"]))
        assert st["polish_solves"] >= st["n_solved"] and st["polish_gated"] >= 0
        assert st["iterations"] == int(np.max(host["iters"]))


@pytest.mark.parametrize("cfg,k", [("c3", 63), ("c3", 64), ("c3", 65), ("c3", 96),
                                   ("c2", 86), ("c2", 87)])
def test_factor_block_widths_around_the_register_layout(cfg, k):
    # K^-1 of a factor block of k + G columns: in registers up to 96 (lanes
    # hold columns lane and lane + 64, waves rows w + 16 t), triangular
    # sweeps beyond; the widths straddle 64 and 96 (c2 adds 10 band columns)
    uni, book = make_config(cfg, 11, N=700, M=2, k=k)
    host, _ = run_gpu(uni, book, rho=5.0)
    for a in range(book.m):
        check_account(uni, book, a, host)


@pytest.mark.parametrize("hw", [1e-4, 1e-3, 5e-3])
def test_tight_sector_bands(hw):
    # ten sector bands of half-width hw around the equal-weight shares: at
    # 1e-4 nearly all bind (a constraint system past eight columns, whose
    # band rows sum to the budget row: dependent, solved with null
    # directions), wider bands leave a few active (the system in LDS)
    uni, book = make_config("c2", 11, N=700, M=3, k=8, band_halfwidth=hw)
    host, _ = run_gpu(uni, book, rho=5.0)
    for a in range(book.m):
        check_account(uni, book, a, host)


def test_one_handle_across_growing_books():
    # a small book, then larger ones (more accounts, more assets) on the same
    # handle: the pinned class staging and the workspaces grow between calls
    from paper_2606_23367_amd.solver import Solver
    s = Solver(0)
    for seed, N, M in ((13, 600, 3), (14, 900, 12), (15, 1300, 20)):
        uni, book = make_config("c3", seed, N=N, M=M, k=8)
        host, st = run_gpu(uni, book, solver=s, rho=5.0)
        assert st["n_solved"] == M
        for a in (0, M // 2, M - 1):
            check_account(uni, book, a, host)


def test_run_to_run_deterministic():
    uni, book = make_config("c3", 4, N=1500, M=6, k=12)
    h1, _ = run_gpu(uni, book, rho=5.0)
    h2, _ = run_gpu(uni, book, rho=5.0)
    assert np.array_equal(h1["w"], h2["w"])
    assert np.array_equal(h1["iters"], h2["iters"])


def test_graph_and_direct_launch_agree():
    uni, book = make_config("c2", 5, N=600, M=5, k=8)
    h1, _ = run_gpu(uni, book, rho=1.0, use_graph=1)
    h2, _ = run_gpu(uni, book, rho=1.0, use_graph=0)
    assert np.array_equal(h1["w"], h2["w"])


def test_batched_equals_one_account_per_launch():
    uni, book = make_config("c3", 6, N=1200, M=5, k=10)
    hb, _ = run_gpu(uni, book, rho=5.0)
    for a in range(book.m):
        ha, _ = run_gpu(uni, subset_accounts(book, [a]), rho=5.0)
        assert ha["status"][0] == hb["status"][a] == 0
        assert np.max(np.abs(ha["w"][0] - hb["w"][a])) <= 1e-9
