"""Invariants of the seeded input generator (it holds none of the sort's arithmetic)."""
import numpy as np

import gen


def test_deterministic_per_seed():
    a = gen.column(100000, 300, dist="zipf", s=1.1)
    b = gen.column(100000, 300, dist="zipf", s=1.1)
    c = gen.column(100000, 300, dist="zipf", s=1.1, seed=gen.default_seed(100000, 300, rep=1))
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)


def test_palette_distinct_and_realised_k():
    x = gen.column(200000, 1000)
    assert np.unique(x).size == 1000
    pal = {gen.palette_value("random", 7, r) for r in range(5000)}
    assert len(pal) == 5000  # the SplitMix64 finaliser is a bijection
    codes = gen.column(50000, 64, palette="codes", dtype=np.uint64)
    assert codes.max() < 64


def test_k_at_least_n_is_all_distinct():
    x = gen.column(10000, 10000)
    assert np.unique(x).size == 10000


def test_zipf_cdf():
    cdf = gen.zipf_cdf(1000, 1.0)
    assert np.all(np.diff(cdf) > 0) and cdf[-1] == 1.0
    # rank 0 is the hottest: its share is 1 / H_1000 (harmonic number)
    h = np.sum(1.0 / np.arange(1, 1001))
    assert abs(cdf[0] - 1.0 / h) < 1e-12
    x = gen.column(400000, 1000, dist="zipf", s=1.0, palette="codes", dtype=np.uint64)
    share0 = np.mean(x == 0)
    assert abs(share0 - 1.0 / h) < 0.005


def test_splitmix_counter_form():
    # output i is the finaliser of seed + (i+1) * golden
    g = 0x9E3779B97F4A7C15
    for i in range(5):
        assert gen.splitmix(123, i) == gen.mix64((123 + (i + 1) * g) % 2**64)


def test_structured_shapes():
    n, k = 50000, 50
    g = gen.column(n, k, dist="grouped", dtype=np.uint64)
    assert np.count_nonzero(g[1:] != g[:-1]) == np.unique(g).size - 1  # one run per value
    runs = gen.column(n, k, dist="runs")
    assert np.count_nonzero(runs[1:] != runs[:-1]) < n // 2
    almost = gen.column(n, k, dist="almost_sorted")
    assert np.unique(almost).size <= k


def test_runs_recipe_mean_length():
    """Run-shaped columns: runs of random length 1..2L-1 (mean L = N / (4K)), one
    palette value per run (neighbouring runs merge when they draw the same value,
    with probability 1/K)."""
    n, k = 1 << 20, 64
    x = gen.column(n, k, dist="runs", dtype=np.uint64)
    boundaries = np.count_nonzero(x[1:] != x[:-1])
    mean_len = n / (boundaries + 1)
    L = n / (4 * k)
    assert 0.85 * L <= mean_len <= 1.3 * L, (mean_len, L)
    assert np.unique(x).size <= k


def test_almost_sorted_recipe_swaps():
    """Almost sorted: the sorted-by-group column with N/100 random transpositions,
    so at most 2% of the positions differ from it."""
    n, k = 200_000, 300
    g = gen.column(n, k, dist="grouped", dtype=np.uint64)
    a = gen.column(n, k, dist="almost_sorted", dtype=np.uint64)
    assert np.array_equal(np.sort(a), np.sort(g))
    assert 0 < np.count_nonzero(a != g) <= 2 * (n // 100)
