"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here re-derives a value with the oracle's own code: expected values
come from a library routine (numpy / Python sorting), brute force, closed
forms worked by hand from the paper's definitions, numbers the paper prints
(tests/golden/paper_values.json), or a Poisson model.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import gen
import oracle
from tests import crafted

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1
U64_MAX = (1 << 64) - 1


# --------------------------------------------------------------------------
# Output and counts: library sort, brute force, invariants (Sec. 3.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.int64, np.uint64])
@pytest.mark.parametrize("n,k,dist,pal", [
    (0, 1, "uniform", "random"), (1, 1, "uniform", "random"), (7, 3, "uniform", "random"),
    (1000, 200, "uniform", "random"), (100000, 200, "zipf", "random"),
    (50000, 50000, "uniform", "random"), (20000, 1000, "uniform", "codes"),
    (30000, 17, "runs", "ap"), (30000, 40, "almost_sorted", "random"),
])
def test_sort_equals_numpy_sort(dtype, n, k, dist, pal):
    x = gen.column(n, k, dist=dist, palette=pal, dtype=dtype)
    y = oracle.sort(x, dtype)
    assert y.dtype == dtype
    np.testing.assert_array_equal(y, np.sort(x, kind="stable"))


@pytest.mark.parametrize("dtype", [np.int64, np.uint64])
def test_counts_equal_unique(dtype):
    x = gen.column(200000, 3000, dist="zipf", s=1.1, dtype=dtype)
    uniq, cnt = oracle.counts(x, dtype)
    u_ref, c_ref = np.unique(x, return_counts=True)
    np.testing.assert_array_equal(uniq, u_ref)
    np.testing.assert_array_equal(cnt, c_ref.astype(np.uint64))
    assert int(cnt.sum()) == x.size
    r = oracle.report(x, dtype)
    assert r["k_exact"] == u_ref.size


def test_bruteforce_small_alphabets():
    """All arrays of length <= 6 over a 5-letter alphabet of extreme values:
    output == Python's sorted(); counts == run lengths; MONOTONE iff sorted.
    """
    alph = {
        np.int64: [I64_MIN, -1, 0, 1, I64_MAX],
        np.uint64: [0, 1, (1 << 63) - 1, 1 << 63, U64_MAX],
    }
    for dtype, letters in alph.items():
        for n in range(0, 7):
            for tup in itertools.product(letters, repeat=n):
                x = np.array(tup, dtype=dtype)
                exp = sorted(tup)
                assert oracle.sort(x, dtype).tolist() == exp
                uniq, cnt = oracle.counts(x, dtype)
                runs = [(k, len(list(g))) for k, g in itertools.groupby(exp)]
                assert uniq.tolist() == [k for k, _ in runs]
                assert cnt.tolist() == [c for _, c in runs]
                r = oracle.report(x, dtype)
                mono = list(tup) == exp
                assert r["path"] == ("MONOTONE" if mono else "SMALL_N")
                assert r["k_exact"] == len(runs)


# --------------------------------------------------------------------------
# IsMonotone and the dispatch order (Alg. 3): crafted T1 / T2
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 2047, 2048, 1000000])
def test_t1_sorted_is_monotone(n):
    x, exp = crafted.t1_sorted(n)
    assert oracle.report(x.view(np.int64))["path"] == "MONOTONE"


def test_t1_signedness():
    # [-1, 0] is nondecreasing in signed order; the same bits in unsigned order
    # are [2^64-1, 0], which is not.
    x = np.array([-1, 0], dtype=np.int64)
    assert oracle.is_monotone(x, np.int64)
    assert not oracle.is_monotone(x.view(np.uint64), np.uint64)
    assert oracle.report(x, np.int64)["path"] == "MONOTONE"
    assert oracle.report(x.view(np.uint64), np.uint64)["path"] == "SMALL_N"


def test_t2_small_n_cut():
    x, _ = crafted.t2_unsorted(2047)
    r = oracle.report(x.view(np.int64))
    assert r["path"] == "SMALL_N" and r["n_samples"] == 0
    x, _ = crafted.t2_unsorted(2048)
    r = oracle.report(x.view(np.int64))
    assert r["path"] != "SMALL_N" and r["stride"] == 2 and r["n_samples"] == 1024


# --------------------------------------------------------------------------
# Chao1 over strided samples (Alg. 2, Eq. chao1): closed forms
# --------------------------------------------------------------------------

def test_estimate_all_equal():
    e = oracle.estimate(np.full(5000, 42, dtype=np.uint64))
    # one distinct value seen 1024 times: u = 1, f1 = f2 = 0, K^ = 1 + 0
    assert e == dict(k_hat=1, u=1, f1=0, f2=0, n_samples=1024, stride=4, saturated=0)


def test_estimate_saturates():
    # stride 4 and 1024 distinct values at the sampled positions: u = s -> K^ = N
    x = np.zeros(4096, dtype=np.uint64)
    x[0::4] = np.arange(1, 1025, dtype=np.uint64)
    e = oracle.estimate(x)
    assert e == dict(k_hat=4096, u=1024, f1=1024, f2=0, n_samples=1024, stride=4, saturated=1)


def test_estimate_all_doubletons():
    # 512 values twice each: u = 512, f1 = 0, f2 = 512 -> K^ = 512 + 0
    x = np.repeat(np.arange(512, dtype=np.uint64) * np.uint64(977), 2)
    e = oracle.estimate(x)
    assert e == dict(k_hat=512, u=512, f1=0, f2=512, n_samples=1024, stride=1, saturated=0)


def test_estimate_f2_zero_blowup():
    # 999 singletons + one value 25 times: u = 1000, f1 = 999, f2 = 0
    # K^ = 1000 + floor(998001 / 2) = 1000 + 499000 = 500000
    x = np.concatenate([np.arange(1, 1000, dtype=np.uint64), np.full(25, 7777, dtype=np.uint64)])
    e = oracle.estimate(x)
    assert e == dict(k_hat=500000, u=1000, f1=999, f2=0, n_samples=1024, stride=1, saturated=0)


def test_estimate_mixed_spectrum():
    # 10 values x1, 6 values x2, 1 value x1002 (1024 samples, stride 1):
    # u = 17, f1 = 10, f2 = 6 -> K^ = 17 + floor(100 / 14) = 17 + 7 = 24
    x = np.concatenate([np.arange(100, 110), np.repeat(np.arange(200, 206), 2),
                        np.full(1002, 5)]).astype(np.uint64)
    e = oracle.estimate(x)
    assert e == dict(k_hat=24, u=17, f1=10, f2=6, n_samples=1024, stride=1, saturated=0)


def test_estimate_small_and_empty():
    assert oracle.estimate(np.zeros(0, dtype=np.uint64)) == dict(
        k_hat=0, u=0, f1=0, f2=0, n_samples=0, stride=1, saturated=0)
    # N = 5 < s: stride 1, every element sampled, never saturated
    e = oracle.estimate(np.array([1, 2, 3, 4, 5], dtype=np.uint64))
    assert e == dict(k_hat=5 + 25 // 2, u=5, f1=5, f2=0, n_samples=5, stride=1, saturated=0)


@pytest.mark.parametrize("n,stride,last", [
    (1023, 1, 1022), (1024, 1, 1023), (2047, 1, 1023), (2048, 2, 2046),
    (3071, 2, 2046), (3072, 3, 3069), (10**6, 976, 976 * 1023),
])
def test_sample_positions(n, stride, last):
    """Samples are x[0], x[stride], ... while i < min(N, 1024*stride).

    Marking exactly those positions with distinct values and everything else with
    one other value gives u = n_samples; changing any other position changes
    nothing; changing a sampled position changes u.
    """
    x = np.zeros(n, dtype=np.uint64)
    pos = np.arange(0, last + 1, stride)
    assert pos.size == min(n, 1024)
    x[pos] = np.arange(1, pos.size + 1, dtype=np.uint64) * np.uint64(3)  # distinct, nonzero
    e = oracle.estimate(x)
    assert e["stride"] == stride and e["n_samples"] == pos.size and e["u"] == pos.size
    y = x.copy()
    others = np.setdiff1d(np.arange(n), pos)
    if others.size:
        y[others] = np.uint64(999999937)
        assert oracle.estimate(y) == e
    z = x.copy()
    z[pos[-1]] = z[pos[0]]  # one sampled value duplicated -> u drops by one
    assert oracle.estimate(z)["u"] == pos.size - 1


def test_estimate_relabelling_invariance():
    x = gen.column(100000, 700, dist="zipf", s=1.0, dtype=np.uint64)
    e = oracle.estimate(x)
    # any bijection of the values (odd multiplier plus offset mod 2^64)
    y = x * np.uint64(0xD1B54A32D192ED03) + np.uint64(12345)
    assert oracle.estimate(y) == e


# --------------------------------------------------------------------------
# Eq. Msize with the paper's worked sizes; Eq. hash closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", GOLDEN["table_M_worked"]["cases"])
def test_table_M_worked_values(case):
    n = 1 << 26  # large enough that the upper clamp bit_ceil(N/4) does not bind
    M = oracle.table_M(case["k_hat"], n)
    assert M == case["M"]
    assert M * GOLDEN["table_M_worked"]["bucket_bytes"] == case["bytes"]


def test_table_M_clamps():
    assert oracle.table_M(1, 10**6) == 8           # 2*1 -> 2, lower clamp 8
    assert oracle.table_M(3, 10**6) == 8           # 6 -> 8
    assert oracle.table_M(5, 10**6) == 16          # 10 -> 16
    assert oracle.table_M(1000, 2048) == 512       # bit_ceil(2000) = 2048 > bit_ceil(512)
    assert oracle.table_M(1000, 2051) == 512       # integer N/4 = 512
    assert oracle.table_M(1000, 2052) == 1024      # N/4 = 513 -> bit_ceil = 1024


def test_hash_constant_and_inverse():
    assert int(GOLDEN["hash_multiplier"]["value_hex"], 16) == crafted.PHI
    assert (crafted.PHI * crafted.PHI_INV) % (1 << 64) == 1


def test_hash_closed_forms():
    # h(1) = top m bits of 0x9E3779B97F4A7C15: 0x9E37 = 1001 1110 0011 0111b
    assert oracle.hash_bucket(1, 512) == 0b100111100          # 316
    assert oracle.hash_bucket(1, 4096) == 0b100111100011       # 2531
    assert oracle.hash_bucket(1, 8) == 0b100
    # 2^63 * odd = 2^63 (mod 2^64): the top bit only -> M/2
    for M in (8, 512, 1 << 20):
        assert oracle.hash_bucket(1 << 63, M) == M // 2
        assert oracle.hash_bucket(0, M) == 0
    rng = np.random.default_rng(11)
    for m in (3, 5, 9, 17, 30):
        for _ in range(50):
            b = int(rng.integers(0, 1 << m))
            assert oracle.hash_bucket(crafted.key_in_bucket(b, m, int(rng.integers(0, 2**62))), 1 << m) == b


def test_dictionary_codes_spread():
    # Codes 0..K-1 under the multiplicative hash (Sec. 4.2): consecutive keys are
    # spread apart (Fibonacci hashing), so K <= M/2 codes never fill a 4-slot
    # bucket.  A progression with step M, which x mod M would send to one bucket,
    # is spread as well: 64 such keys into M = 1024 buckets spill nothing.
    for K in (200, 1000, 5000):
        M = 1 << (2 * K - 1).bit_length()
        assert oracle.spill(np.arange(K, dtype=np.uint64), M) == 0
    prog = np.arange(0, 64 * 1024, 1024, dtype=np.uint64)  # 64 keys, step M
    assert oracle.spill(prog, 1024) == 0


# --------------------------------------------------------------------------
# Bucket simulation and guard (Alg. 1 + RLE, Alg. 4)
# --------------------------------------------------------------------------

def test_spill_first_four_claim():
    M, m = 8, 3
    ks = [crafted.key_in_bucket(5, m, 100 + i) for i in range(7)]
    # first-occurrence order k0..k6, counts 1..7: k4, k5, k6 spill -> 5 + 6 + 7
    seq = []
    for i, k in enumerate(ks):
        seq += [k] * (i + 1)
    assert oracle.spill(np.array(seq, dtype=np.uint64), M) == 18
    # later occurrences of early keys interleaved after the spilled ones: no change
    seq2 = seq + [ks[0], ks[4], ks[1], ks[6]]
    assert oracle.spill(np.array(seq2, dtype=np.uint64), M) == 18 + 2
    # four keys per bucket in every bucket: nothing spills
    full = [crafted.key_in_bucket(b, m, 7 * i) for b in range(8) for i in range(4)]
    assert oracle.spill(np.array(full * 3, dtype=np.uint64), M) == 0


def test_spill_runs_counted_in_elements():
    M, m = 8, 3
    ks = [crafted.key_in_bucket(2, m, 50 + i) for i in range(5)]
    x = np.array(ks[:4] + [ks[4]] * 100 + ks[:4], dtype=np.uint64)
    assert oracle.spill(x, M) == 100


@pytest.mark.parametrize("name", list(crafted.all_cases().keys()))
def test_crafted_reports(name):
    x, exp = crafted.all_cases()[name]
    for dtype in (np.int64, np.uint64):
        r = oracle.report(x.view(dtype), dtype)
        for key, val in exp.items():
            assert r[key] == val, (name, dtype, key, r[key], val)


def test_poisson_overflow_rate():
    """K = 2^20 distinct random keys into M = 2^21 buckets (mean fill 0.5, cap 4):
    expected spilled keys = M * E[(X - 4)^+] for X ~ Poisson(0.5).  The paper's
    P(X >= 5) ~ 1.7e-4 is the leading term of that sum.
    """
    lam, cap = GOLDEN["poisson_overflow"]["mean_fill"], GOLDEN["poisson_overflow"]["cap"]
    p5 = math.exp(-lam) * sum(lam ** k / math.factorial(k) for k in range(cap + 1, 40))
    assert abs(p5 - GOLDEN["poisson_overflow"]["p_overflow"]) < 0.05e-4
    excess = math.exp(-lam) * sum((k - cap) * lam ** k / math.factorial(k) for k in range(cap + 1, 40))
    M = 1 << 21
    x = gen.column(1 << 20, 1 << 20, dtype=np.uint64)  # K >= n: n distinct random values
    assert np.unique(x).size == x.size
    sp = oracle.spill(x, M)
    mean = M * excess
    assert abs(sp - mean) < 6 * math.sqrt(mean * 1.5), (sp, mean)


def test_zipf_sweep_reports_main_path():
    # Zipf(1.1) with K = 1e4 at N = 2e6: Chao1 underestimates K (Sec. 2.4's
    # singleton/doubleton signal is weak under skew) but stays on the main path.
    x = gen.column(2_000_000, 10_000, dist="zipf", s=1.1)
    r = oracle.report(x)
    assert r["path"] == "MAIN" and r["k_hat"] < r["k_exact"]
    assert r["table_M"] == oracle.table_M(r["k_hat"], x.size)


def test_std_sort_baseline_is_a_sort():
    """The std::sort baseline the bench reports beside the oracle sorts (numpy agrees),
    extremes and duplicates included."""
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.integers(-2**63, 2**63 - 1, size=5000, dtype=np.int64),
                        np.array([-2**63, 2**63 - 1, 0, -1, 0, -2**63], dtype=np.int64)])
    assert np.array_equal(oracle.std_sort_i64(x), np.sort(x))
    assert oracle.std_sort_i64(np.empty(0, dtype=np.int64)).size == 0


# ---- float64 keys in IEEE 754 totalOrder ------------------------------------

def _f64(bits):
    return np.array(bits, dtype=np.uint64).view(np.float64)


def test_f64_total_order_special_values():
    """The order that IEEE 754-2008 (Sec. 5.10, totalOrder) fixes for signed zeros,
    infinities, subnormals and NaNs of either sign."""
    neg_nan, pos_nan = 0xFFF8000000000000, 0x7FF8000000000000
    neg_nan_payload = 0xFFF8000000000001   # larger payload: further below
    pos_nan_payload = 0x7FF8000000000001   # larger payload: further above
    want_bits = [neg_nan_payload, neg_nan, 0xFFF0000000000000,               # -NaN(1) < -NaN < -inf
                 np.float64(-1.5).view(np.uint64), 0x8000000000000001,       # -1.5 < -min subnormal
                 0x8000000000000000, 0x0000000000000000,                     # -0 < +0
                 0x0000000000000001, np.float64(2.0).view(np.uint64),        # +min subnormal < 2
                 0x7FF0000000000000, pos_nan, pos_nan_payload]               # +inf < +NaN < +NaN(1)
    want = np.array(want_bits, dtype=np.uint64)
    rng = np.random.default_rng(3)
    x = want[rng.permutation(want.size)]
    got = oracle.sort(x.view(np.float64), np.float64).view(np.uint64)
    assert np.array_equal(got, want)
    assert oracle.is_monotone(want.view(np.float64), np.float64)
    assert not oracle.is_monotone(want[::-1].copy().view(np.float64), np.float64)


def test_f64_sort_matches_numpy_on_ordinary_values():
    """Away from zeros and NaNs totalOrder is the numeric order, which numpy's sort
    gives; repeated values keep their multiplicities."""
    rng = np.random.default_rng(11)
    pal = rng.normal(size=300) * 10.0 ** rng.uniform(-300, 300, size=300)
    pal = np.concatenate([pal, [np.inf, -np.inf, 5e-324, -5e-324]])
    x = pal[rng.integers(0, pal.size, size=20_000)]
    assert np.array_equal(oracle.sort(x, np.float64), np.sort(x))
    u, c = oracle.counts(x, np.float64)
    nu, nc = np.unique(x, return_counts=True)
    assert np.array_equal(u, nu) and np.array_equal(c, nc.astype(np.uint64))


def test_f64_zeros_and_nans_are_distinct_keys():
    """Equality is on the bit pattern: -0 and +0 count apart, NaNs with different
    payloads count apart."""
    bits = np.array([0x0, 0x8000000000000000, 0x0, 0x7FF8000000000000, 0x7FF8000000000002,
                     0x7FF8000000000000, 0xFFF8000000000000], dtype=np.uint64)
    u, c = oracle.counts(bits.view(np.float64), np.float64)
    assert list(u.view(np.uint64)) == [0xFFF8000000000000, 0x8000000000000000, 0x0,
                                       0x7FF8000000000000, 0x7FF8000000000002]
    assert list(c) == [1, 1, 2, 2, 1]


def test_f64_report_follows_the_bits():
    """Estimate, tiny check, bucket table and spill act on bit patterns, so a
    float64 column reports what the same bits report as uint64 (the order matters
    only to the monotone test)."""
    rng = np.random.default_rng(5)
    for n, k in ((50_000, 6), (60_000, 900), (40_000, 30_000)):
        pal = rng.normal(size=k)
        x = pal[rng.integers(0, k, size=n)]
        rf = oracle.report(x, np.float64)
        ru = oracle.report(x.view(np.uint64), np.uint64)
        assert rf == ru, (n, k)
    s = np.sort(rng.normal(size=5000))
    assert oracle.report(s, np.float64)["path"] == "MONOTONE"
    assert oracle.report(-s, np.float64)["path"] != "MONOTONE"


# --------------------------------------------------------------------------
# 32-bit keys (Sec. 4.2's int32 specialization): sort, counts, Eq. Msize with
# cap 8, buckets of eight keys, the estimate on the 32-bit patterns
# --------------------------------------------------------------------------

I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1


def _col32(n, k, seed, signed):
    rng = np.random.default_rng(seed)
    if signed:
        pal = rng.integers(I32_MIN, I32_MAX, size=k, endpoint=True, dtype=np.int64).astype(np.int32)
    else:
        pal = rng.integers(0, 1 << 32, size=k, dtype=np.uint64).astype(np.uint32)
    return pal[rng.integers(0, k, size=n)]


@pytest.mark.parametrize("signed", [True, False])
@pytest.mark.parametrize("n,k", [(0, 1), (1, 1), (9, 4), (5000, 200), (100_000, 3000), (40_000, 40_000)])
def test_sort32_equals_numpy_sort(signed, n, k):
    dt = np.int32 if signed else np.uint32
    x = _col32(n, k, n + k, signed)
    y = oracle.sort(x, dt)
    assert y.dtype == dt and np.array_equal(y, np.sort(x, kind="stable"))
    u, c = oracle.counts(x, dt)
    uu, cc = np.unique(x, return_counts=True)
    assert np.array_equal(u, uu) and np.array_equal(c, cc.astype(np.uint64))
    assert int(c.sum()) == n
    assert oracle.is_monotone(y, dt) and (n < 2 or not oracle.is_monotone(np.sort(x)[::-1].copy(), dt)
                                          or np.unique(x).size == 1)


def test_bruteforce_small_alphabets_32():
    alph = {np.int32: [I32_MIN, -1, 0, 1, I32_MAX], np.uint32: [0, 1, (1 << 31) - 1, 1 << 31, (1 << 32) - 1]}
    for dt, vals in alph.items():
        for length in range(0, 6):
            for combo in itertools.product(vals, repeat=length):
                x = np.array(combo, dtype=dt)
                assert oracle.sort(x, dt).tolist() == sorted(combo), (dt, combo)
                u, c = oracle.counts(x, dt)
                assert u.tolist() == sorted(set(combo)), (dt, combo)
                assert c.tolist() == [combo.count(v) for v in sorted(set(combo))]
                assert oracle.is_monotone(x, dt) == (list(combo) == sorted(combo))


def test_signedness_32():
    # the same bits order as signed or unsigned 32-bit integers
    x = np.array([0xFFFFFFFF, 0, 0x80000000, 5], dtype=np.uint32)
    assert oracle.sort(x, np.uint32).tolist() == [0, 5, 0x80000000, 0xFFFFFFFF]
    assert oracle.sort(x.view(np.int32), np.int32).tolist() == [I32_MIN, -1, 0, 5]
    assert oracle.is_monotone(np.array([-1, 0], dtype=np.int32), np.int32)
    assert not oracle.is_monotone(np.array([0xFFFFFFFF, 0], dtype=np.uint32), np.uint32)


def test_table_M_cap8_closed_forms():
    cap = GOLDEN["bucket_cap_32"]["cap"]
    assert cap == 8 and GOLDEN["bucket_cap_32"]["cap_64"] == 4
    n = 1 << 26
    # M = bit_ceil(8 K^ / 8) = bit_ceil(K^): half the 64-bit table of the same estimate
    for kh, m in ((200, 256), (1000, 1024), (4000, 4096), (10_000, 16_384), (1_000_000, 1 << 20)):
        assert oracle.table_M(kh, n, cap=8) == m
        assert oracle.table_M(kh, n, cap=4) == 2 * m
    assert oracle.table_M(1, 10**6, cap=8) == 8       # lower clamp
    assert oracle.table_M(7, 10**6, cap=8) == 8
    assert oracle.table_M(9, 10**6, cap=8) == 16
    assert oracle.table_M(1000, 2048, cap=8) == 256   # upper clamp bit_ceil(N/8) = 256
    assert oracle.table_M(1000, 2055, cap=8) == 256   # integer N/8 = 256
    assert oracle.table_M(1000, 2056, cap=8) == 512   # N/8 = 257 -> 512


def _keys32_in_bucket(b, M, count, start=1):
    """The first `count` 32-bit values from `start` whose Eq. hash (on the
    zero-extended pattern) lands in bucket b of M, found by scanning."""
    out, v = [], start
    while len(out) < count:
        if oracle.hash_bucket(v, M) == b:
            out.append(v)
        v += 1
    return out


def test_spill_cap8_first_eight_claim():
    M = 8
    ks = _keys32_in_bucket(3, M, 11)
    # first-occurrence order k0..k10 with counts 1..11: k8, k9, k10 spill with cap 8
    seq = []
    for i, k in enumerate(ks):
        seq += [k] * (i + 1)
    x = np.array(seq, dtype=np.uint64)
    assert oracle.spill(x, M, cap=8) == 9 + 10 + 11
    # the same keys with cap 4: k4..k10 spill
    assert oracle.spill(x, M, cap=4) == sum(range(5, 12))
    # eight keys in every bucket: nothing spills with cap 8
    full = [k for b in range(M) for k in _keys32_in_bucket(b, M, 8)]
    assert oracle.spill(np.array(full * 2, dtype=np.uint64), M, cap=8) == 0


def test_report32_reads_patterns_and_cap8():
    """A 32-bit column's estimate is the estimate of its zero-extended patterns;
    M and the spill come from buckets of eight: a crafted column where 12 keys share
    one of M = 8 buckets spills exactly the elements of keys 9..12."""
    M = 8
    ks = _keys32_in_bucket(6, M, 12, start=1 << 31)  # patterns with bit 31 set: negative as int32
    # N = 2560 > 2048, stride 2; every sampled (even) position holds ks[0]: u = 1, K^ = 1
    n = 2560
    x = np.full(n, ks[0], dtype=np.uint64)
    odd = np.arange(1, n, 2)
    for i, k in enumerate(ks[1:]):
        x[odd[i * 100:(i + 1) * 100]] = k  # 100 copies each, in first-occurrence order
    x32 = x.astype(np.uint32)
    for dt in (np.uint32, np.int32):
        r = oracle.report(x32.view(dt), dt)
        assert (r["k_hat"], r["u"], r["f1"], r["f2"], r["n_samples"], r["stride"]) == (1, 1, 0, 0, 1024, 2)
        assert r["tiny_miss"] == 1 and r["table_M"] == 8, r
        assert r["spill_elems"] == 4 * 100, r          # keys 9..12 (indices 8..11), 100 each
        assert r["path"] == "MAIN" and r["k_exact"] == 12
    # with 64-bit keys of the same values the buckets hold four: keys 5..12 spill
    r64 = oracle.report(x, np.uint64)
    assert r64["spill_elems"] == 8 * 100 and r64["table_M"] == 8


# ---- key-value sort (stable; payloads move with their keys) -----------------

def _order_key_f64(bits):
    """totalOrder as an unsigned order: flip every bit of a pattern with the sign
    set, flip only the sign bit otherwise (IEEE 754-2008, Sec. 5.10)."""
    b = bits.view(np.uint64)
    neg = (b >> np.uint64(63)) != 0
    return np.where(neg, ~b, b ^ np.uint64(1 << 63))


@pytest.mark.parametrize("dtype", [np.int64, np.uint64, np.int32, np.uint32, np.float64])
@pytest.mark.parametrize("n,k", [(1, 1), (50_000, 3), (50_000, 700), (30_000, 30_000)])
def test_sort_kv_equals_numpy_stable_argsort(dtype, n, k):
    """The key-value sort is numpy's stable argsort applied to keys and payloads."""
    rng = np.random.default_rng(n + k)
    if dtype == np.float64:
        pal = rng.normal(size=k) * 10.0 ** rng.uniform(-20, 20, size=k)
        x = pal[rng.integers(0, k, size=n)]
        order = np.argsort(_order_key_f64(x), kind="stable")
    else:
        info = np.iinfo(dtype)
        pal = rng.integers(info.min, info.max, size=k, dtype=dtype, endpoint=True)
        x = pal[rng.integers(0, k, size=n)]
        order = np.argsort(x, kind="stable")
    v = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64, endpoint=True)
    y, w = oracle.sort_kv(x, v, dtype)
    assert np.array_equal(y.view(np.uint8), x[order].view(np.uint8))
    assert np.array_equal(w, v[order])


def test_sort_kv_bruteforce_small_alphabets():
    """Every sequence of up to 7 keys over three values (one of them negative),
    payloads = positions: the keys equal the keys-only sort, each payload points at
    an input position holding its key, and within equal keys the positions rise."""
    for dtype in (np.int64, np.int32, np.uint32):
        alphabet = np.array([-3, 0, 5], dtype=np.int64).astype(dtype)
        for L in range(0, 8):
            for combo in itertools.product(range(3), repeat=L):
                x = alphabet[list(combo)] if L else np.zeros(0, dtype=dtype)
                v = np.arange(L, dtype=np.uint64)
                y, w = oracle.sort_kv(x, v, dtype)
                assert np.array_equal(y, oracle.sort(x, dtype))
                assert sorted(w.tolist()) == list(range(L))
                assert np.array_equal(x[w.astype(np.int64)], y)
                for i in range(1, L):
                    if y[i] == y[i - 1]:
                        assert w[i] > w[i - 1]


def test_sort_kv_f64_bits_are_keys():
    """float64 keys: -0 and +0, and NaNs with different payloads, are different keys
    in totalOrder; payloads follow them."""
    bits = np.array([0x0000000000000000, 0x8000000000000000, 0x7FF8000000000001, 0x7FF8000000000000,
                     0x8000000000000000, 0xFFF0000000000000, 0x0000000000000000], dtype=np.uint64)
    v = np.arange(bits.size, dtype=np.uint64) * np.uint64(10)
    y, w = oracle.sort_kv(bits.view(np.float64), v, np.float64)
    assert y.view(np.uint64).tolist() == [0xFFF0000000000000, 0x8000000000000000, 0x8000000000000000,
                                          0x0000000000000000, 0x0000000000000000, 0x7FF8000000000000,
                                          0x7FF8000000000001]
    assert w.tolist() == [50, 10, 40, 0, 60, 30, 20]


def test_sort_kv_planted_mistakes_are_caught():
    """The pins above fail for the mistakes a key-value sort can plausibly make:
    an unstable order within a key and payloads left in input order."""
    rng = np.random.default_rng(5)
    x = rng.integers(0, 4, size=200).astype(np.int64)
    v = np.arange(200, dtype=np.uint64)
    y, w = oracle.sort_kv(x, v, np.int64)
    order = np.argsort(x, kind="stable")
    unstable = np.argsort(x, kind="quicksort")[::-1]
    unstable = unstable[np.argsort(x[unstable], kind="stable")]  # keys sorted, ties reversed
    assert not np.array_equal(v[unstable], v[order])
    assert np.array_equal(w, v[order])
    assert not np.array_equal(w, v)
