"""Hand-built inputs that force each dispatcher branch and guard boundary.

Every builder returns ``(x, expected)`` where ``x`` is a uint64 numpy array
(bit patterns; view it as int64 for signed order) and ``expected`` is a dict of
report fields derived by hand from the paper's rules (Alg. 2, Alg. 3, Alg. 1,
Eq. hash, Eq. Msize, Alg. 4).  The derivation of each number is in the comment
beside it.  The GPU parity tests reuse the same inputs and compare against the
oracle.
"""
import numpy as np

MASK = (1 << 64) - 1
PHI = 0x9E3779B97F4A7C15          # Eq. hash multiplier
PHI_INV = 0xF1DE83E19937733D      # its inverse mod 2^64 (checked in the tests)
INT64_MIN_BITS = 1 << 63
UINT64_MAX = MASK


def key_in_bucket(b, m, salt):
    """A key whose Eq. hash bucket at M = 2^m is ``b``.

    x = y * PHI_INV gives x * PHI = y (mod 2^64), whose top m bits are b.
    """
    low = salt & ((1 << (64 - m)) - 1)
    y = (b << (64 - m)) | low
    return (y * PHI_INV) & MASK


def _rng(seed):
    return np.random.default_rng(seed)


def t1_sorted(n, seed=1):
    """Sorted input with duplicates -> MONOTONE whatever N is."""
    r = _rng(seed)
    x = np.sort(r.integers(-50, 50, size=n, dtype=np.int64)).view(np.uint64)
    return x, {"path": "MONOTONE"}


def t2_unsorted(n, seed=2):
    r = _rng(seed)
    x = r.integers(0, 10, size=n, dtype=np.int64)
    if n >= 2:
        x[0], x[1] = 5, 3  # guarantee an inversion
    return x.view(np.uint64), {"path": "SMALL_N" if n < 2048 else None}


def t3_tiny(values=None):
    """u = 8, f1 = f2 = 0 -> K^ = 8 + 0 = 8 -> TINY (K^ <= 8 and u <= 8).

    N = 4096, stride = 4; x[i] = v[(i // 4) % 8] puts every value at 128 sampled
    positions, and the input holds no other value.
    """
    if values is None:
        values = [INT64_MIN_BITS, UINT64_MAX, 0, 1, (1 << 63) - 1, 12345, 2**40 + 7, 99]
    v = np.array(values, dtype=np.uint64)
    n = 4096
    x = v[(np.arange(n) // 4) % 8]
    exp = dict(k_hat=8, u=8, f1=0, f2=0, n_samples=1024, stride=4, saturated=0,
               path="TINY", tiny_miss=0, table_M=0, spill_elems=0, k_exact=8)
    return x, exp


def t3_not_tiny():
    """u = 8 with f1 = 2, f2 = 0 -> K^ = 8 + 2*2/(2*1) = 10 -> not tiny -> MAIN.

    M = bit_ceil(2*10) = 32 (below bit_ceil(4096/4) = 1024); the 8 keys sit in 8
    different buckets, so nothing spills.
    """
    n = 4096
    keys = [key_in_bucket(b, 5, 0x1234 + 97 * b) for b in range(8)]
    samp = np.empty(1024, dtype=np.uint64)
    samp[0], samp[1] = keys[6], keys[7]          # the two singletons
    samp[2:] = np.array(keys[:6], dtype=np.uint64)[np.arange(1022) % 6]  # ~170 each
    x = np.full(n, keys[0], dtype=np.uint64)
    x[0::4] = samp
    exp = dict(k_hat=10, u=8, f1=2, f2=0, n_samples=1024, stride=4, saturated=0,
               path="MAIN", tiny_miss=0, table_M=32, spill_elems=0, k_exact=8)
    return x, exp


def t4_tiny_miss():
    """Samples see 3 values (K^ = 3 -> tiny); index 1 (unsampled, stride 4) holds a
    4th value -> the sum check fails -> tiny_miss = 1 -> main path with K^ = 3:
    M = max(8, bit_ceil(6)) = 8; 4 distinct keys cannot overfill a bucket -> spill 0.
    """
    n = 4096
    a, b, c, d = INT64_MIN_BITS, 7, UINT64_MAX, 2**62 + 3
    x = np.full(n, a, dtype=np.uint64)
    x[0::4] = np.array([a, b, c], dtype=np.uint64)[np.arange(1024) % 3]
    x[1] = d
    exp = dict(k_hat=3, u=3, f1=0, f2=0, n_samples=1024, stride=4, saturated=0,
               path="MAIN", tiny_miss=1, table_M=8, spill_elems=0, k_exact=4)
    return x, exp


def _blowup_column(n):
    """Sampled positions (stride 3): 62 singletons + one value 962 times.

    u = 63, f1 = 62, f2 = 0 -> K^ = 63 + 62^2 / 2 = 63 + 1922 = 1985.
    """
    stride = n // 1024
    assert stride == 3
    singles = [key_in_bucket(b, 10, 0xABC + b) for b in range(1, 63)]
    rep = key_in_bucket(900, 10, 0x77)
    x = np.full(n, rep, dtype=np.uint64)
    samp = np.full(1024, rep, dtype=np.uint64)
    samp[:62] = np.array(singles, dtype=np.uint64)
    x[0:3072:3] = samp
    return x


def t5_boundary_main():
    """2 K^ = N: N = 3970, K^ = 1985 -> 2K^ > N is false -> MAIN.

    M = min(bit_ceil(3970), bit_ceil(3970 // 4 = 992)) = 1024; the 63 keys sit in
    63 different buckets of M = 1024 -> spill 0.
    """
    x = _blowup_column(3970)
    exp = dict(k_hat=1985, u=63, f1=62, f2=0, n_samples=1024, stride=3, saturated=0,
               path="MAIN", tiny_miss=0, table_M=1024, spill_elems=0, k_exact=63)
    return x, exp


def t5_boundary_high_k():
    """2 K^ = N + 1: N = 3969 (stride still 3), K^ = 1985 -> HIGH_K."""
    x = _blowup_column(3969)
    exp = dict(k_hat=1985, u=63, f1=62, f2=0, n_samples=1024, stride=3, saturated=0,
               path="HIGH_K", tiny_miss=0, table_M=0, spill_elems=0, k_exact=63)
    return x, exp


def t6_all_distinct(n=4096, seed=6):
    """1024 distinct samples -> u = s = 1024 -> saturated, K^ = N -> HIGH_K."""
    r = _rng(seed)
    x = r.permutation(np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B1) + np.uint64(5))
    exp = dict(k_hat=n, u=1024, f1=1024, f2=0, n_samples=1024, stride=n // 1024, saturated=1,
               path="HIGH_K", tiny_miss=0, table_M=0, spill_elems=0, k_exact=n)
    return x, exp


def _guard_frame(n):
    """N in {8192, 8193}: stride 8, 1024 samples.  The sampled positions hold 16
    keys, 64 times each, in buckets 1..16 of M = 32 -> u = 16, f1 = f2 = 0,
    K^ = 16 -> M = max(8, min(bit_ceil(32), bit_ceil(N//4 = 2048))) = 32.
    """
    assert n // 1024 == 8
    sampled = [key_in_bucket(b, 5, 0x5000 + b) for b in range(1, 17)]
    x = np.full(n, sampled[0], dtype=np.uint64)
    pos = np.arange(0, 8192, 8)
    x[pos] = np.array(sampled, dtype=np.uint64)[np.arange(1024) % 16]
    free = np.setdiff1d(np.arange(n), pos)  # unsampled positions in order
    return x, free


def t7_guard(n, spill):
    """Six keys of bucket 20: k1..k4 occur first and claim the four slots; k5 and
    k6 then find the bucket full -> |spill| = c5 + c6 = ``spill``.
    Guard fires iff 2*spill > N (Alg. 4).
    """
    x, free = _guard_frame(n)
    ks = [key_in_bucket(20, 5, 0x9000 + i) for i in range(6)]
    c5 = spill // 2
    c6 = spill - c5
    seq = ks[:4] + [ks[4]] * c5 + [ks[5]] * c6
    assert len(seq) <= free.size
    x[free[:len(seq)]] = np.array(seq, dtype=np.uint64)
    path = "GUARD" if 2 * spill > n else "MAIN"
    exp = dict(k_hat=16, u=16, f1=0, f2=0, n_samples=1024, stride=8, saturated=0,
               path=path, tiny_miss=0, table_M=32, spill_elems=spill, k_exact=22)
    return x, exp


def t8_order_decides(order):
    """Five keys of bucket 20 with counts {4100, 1, 1, 1, 1}; which one spills
    depends only on first-occurrence order (N = 8192, N/2 = 4096):
      'big_first':  big, s1..s4    -> s4 is 5th -> spill 1    -> MAIN
      'big_last':   s1..s4, big    -> big is 5th -> spill 4100 -> GUARD
      'big_fourth': s1, s2, s3, big (one), s4, rest of big -> s4 is 5th -> spill 1
    """
    n = 8192
    x, free = _guard_frame(n)
    big = key_in_bucket(20, 5, 0xB16)
    sm = [key_in_bucket(20, 5, 0x5A11 + i) for i in range(4)]
    if order == "big_first":
        seq = [big] * 4100 + sm
        spill = 1
    elif order == "big_last":
        seq = sm + [big] * 4100
        spill = 4100
    else:
        seq = sm[:3] + [big] + [sm[3]] + [big] * 4099
        spill = 1
    x[free[:len(seq)]] = np.array(seq, dtype=np.uint64)
    path = "GUARD" if 2 * spill > n else "MAIN"
    exp = dict(k_hat=16, u=16, f1=0, f2=0, n_samples=1024, stride=8, saturated=0,
               path=path, tiny_miss=0, table_M=32, spill_elems=spill, k_exact=21)
    return x, exp


def t9_tiny_miss_guard():
    """N = 4096, stride 4: every sampled position holds A (u = 1, K^ = 1 -> tiny);
    the 3072 unsampled positions hold distinct keys, 384 per bucket of M = 8 ->
    tiny miss -> main with K^ = 1 -> M = max(8, bit_ceil(2)) = 8.  A (index 0)
    takes one slot of its bucket; the other 31 slots go to the first keys of each
    bucket; the remaining 3072 - 31 = 3041 elements spill; 2*3041 > 4096 -> GUARD.
    """
    n = 4096
    a = key_in_bucket(3, 3, 0xAAAA)
    x = np.full(n, a, dtype=np.uint64)
    free = np.setdiff1d(np.arange(n), np.arange(0, n, 4))
    others = [key_in_bucket(i % 8, 3, 0x10000 + i) for i in range(3072)]
    x[free] = np.array(others, dtype=np.uint64)
    exp = dict(k_hat=1, u=1, f1=0, f2=0, n_samples=1024, stride=4, saturated=0,
               path="GUARD", tiny_miss=1, table_M=8, spill_elems=3041, k_exact=3073)
    return x, exp


def all_cases():
    """Every crafted case with a full expected report."""
    return {
        "t3_tiny": t3_tiny(),
        "t3_not_tiny": t3_not_tiny(),
        "t4_tiny_miss": t4_tiny_miss(),
        "t5_main": t5_boundary_main(),
        "t5_high_k": t5_boundary_high_k(),
        "t6_all_distinct": t6_all_distinct(),
        "t7_even_nofire": t7_guard(8192, 4096),
        "t7_even_fire": t7_guard(8192, 4097),
        "t7_odd_nofire": t7_guard(8193, 4096),
        "t7_odd_fire": t7_guard(8193, 4097),
        "t8_big_first": t8_order_decides("big_first"),
        "t8_big_last": t8_order_decides("big_last"),
        "t8_big_fourth": t8_order_decides("big_fourth"),
        "t9_tiny_miss_guard": t9_tiny_miss_guard(),
    }
