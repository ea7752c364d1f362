"""GPU parity for 32-bit keys (int32 and uint32 columns) against the CPU oracle.

The 32-bit path keeps the keys at their 4-byte width in HBM through the count, the
emit and the radix passes; the hash and the tables work on the zero-extended bit
pattern, and Eq. Msize takes eight keys per bucket.  Every comparison is bit-exact:
the sorted output, the distinct keys (at 32 bits) and counts, and every report
field.
"""
import ctypes

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

PHI = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_25040_amd as cafs
    return cafs.Context(0)


def col32(n, k, dist="uniform", s=1.1, palette="random", seed=None):
    """A seeded column of 32-bit keys: the low halves of the 64-bit generator's
    values (dictionary codes stay 0..K-1)."""
    x = gen.column(n, k, dist=dist, s=s, palette=palette, seed=seed, dtype=np.uint64)
    return (x & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def run_gpu(ctx, x32, unsigned, counts=True, shift_in=0, shift_out=0, inplace=False):
    """Sort a uint32 bit-pattern array on the GPU as int32 (or uint32 when
    ``unsigned``); shifts of one key misalign the buffers to 4 bytes."""
    import paper_2605_25040_amd as cafs
    n = x32.size
    buf = torch.empty(n + 2, dtype=torch.int32, device="cuda:0")
    buf[shift_in:shift_in + n].copy_(torch.from_numpy(x32.view(np.int32).copy()))
    x = buf[shift_in:shift_in + n]
    if inplace:
        out = x
    else:
        obuf = torch.empty(n + 2, dtype=torch.int32, device="cuda:0")
        out = obuf[shift_out:shift_out + n]
    out, rep, uq, ct = ctx.sort(x, unsigned=unsigned, out=out, counts=counts)
    torch.cuda.synchronize()
    r = cafs.parse_report(rep)
    dt = np.uint32 if unsigned else np.int32
    y = out.cpu().numpy().view(dt)
    if counts:
        k = r["k_exact"]
        u = uq[:k].cpu().numpy().view(dt)
        c = ct[:k].cpu().numpy().view(np.uint64)
    else:
        u = c = None
    return y, r, u, c


def check(ctx, x32, unsigned, label="", **kw):
    dt = np.uint32 if unsigned else np.int32
    x = x32.view(dt)
    y, r, u, c = run_gpu(ctx, x32, unsigned, **kw)
    want = oracle.sort(x, dt)
    assert np.array_equal(y, want), "%s: sorted output differs" % label
    ro = oracle.report(x, dt)
    for f in oracle.REPORT_FIELDS:
        assert r[f] == ro[f], "%s: report field %s gpu=%r oracle=%r" % (label, f, r[f], ro[f])
    if u is not None:
        uo, co = oracle.counts(x, dt)
        assert np.array_equal(u, uo), "%s: distinct keys differ" % label
        assert np.array_equal(c, co), "%s: counts differ" % label
    return ro


SEEDED = [
    # n, K, dist, palette, path the oracle takes
    (5000, 200, "uniform", "random", "MAIN"),
    (131_072 + 123, 200, "uniform", "random", "MAIN"),
    (200_000, 1000, "zipf", "random", "MAIN"),
    (300_001, 10_000, "uniform", "random", "MAIN"),      # K > 8192: pair sort
    (100_000, 100_000, "uniform", "random", "HIGH_K"),
    (1_000_000, 200, "uniform", "random", "MAIN"),
    (1_000_000, 4, "uniform", "random", "TINY"),
    (1_000_000, 8, "zipf", "random", "TINY"),
    (400_000, 1000, "uniform", "codes", "MAIN"),
    (200_000, 300, "grouped", "random", None),
    (200_000, 64, "runs", "random", None),
    (60_000, 30_000, "zipf", "random", None),
    (1 << 23, 10_000, "zipf", "random", "MAIN"),
    (1 << 23, 20_000, "uniform", "random", "MAIN"),
    (2_000_000, 1_700, "uniform", "random", "MAIN"),
    (2_000_000, 1_900, "uniform", "random", "MAIN"),
    (1 << 24, 10_000, "uniform", "random", "MAIN"),       # hash partitions
    (1 << 24, 100_000, "uniform", "codes", "MAIN"),
    (1 << 22, 300_000, "zipf", "random", None),           # spill list and fold
    (2_000_000, 200_000, "zipf", "random", None),
    (3_000_000, 3_000_000, "zipf", "random", None),
]


@pytest.mark.parametrize("unsigned", [False, True])
@pytest.mark.parametrize("n,k,dist,pal,path", SEEDED)
def test_seeded_columns32(ctx, n, k, dist, pal, path, unsigned):
    x = col32(n, k, dist=dist, palette=pal)
    ro = check(ctx, x, unsigned, label="%s n=%d k=%d" % (dist, n, k))
    if path is not None:
        assert ro["path"] == path, ro


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 64, 2047, 2048, 2049, 4095, 4097, 8193, 9000])
@pytest.mark.parametrize("unsigned", [False, True])
def test_small_and_ragged32(ctx, n, unsigned):
    rng = np.random.default_rng(n + 32)
    x = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32) % np.uint32(max(1, n // 3 + 1))
    check(ctx, x, unsigned, label="n=%d" % n)


EXTREMES = np.array([0x80000000, 0x7FFFFFFF, 0, 1, 0xFFFFFFFF, 0xFFFFFFFE, 0x80000001, 12345], dtype=np.uint32)


@pytest.mark.parametrize("unsigned", [False, True])
@pytest.mark.parametrize("n,k", [(4096, 8), (1_000_000, 8), (1_000_000, 200), (300_000, 20_000),
                                 (50_000, 50_000), (100_000, 1)])
def test_extreme_values_every_path32(ctx, n, k, unsigned):
    """The sign bit, all-ones and zero among the keys of each path (tiny, main,
    pair sort, high K, a single key)."""
    rng = np.random.default_rng(n * 7 + k)
    pal = np.concatenate([EXTREMES, rng.integers(0, 1 << 32, size=max(0, k - 8), dtype=np.uint64)
                          .astype(np.uint32)])[:k]
    x = pal[rng.integers(0, k, size=n)]
    check(ctx, x, unsigned, label="extremes n=%d k=%d" % (n, k))


@pytest.mark.parametrize("shift_in,shift_out", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("n,k", [(1_000_001, 200), (1 << 22, 300_000), (500_000, 500_000), (1_000_000, 4)])
def test_misaligned_by_four_bytes(ctx, shift_in, shift_out, n, k):
    x = col32(n, k, dist="zipf")
    check(ctx, x, False, label="misaligned", shift_in=shift_in, shift_out=shift_out)


@pytest.mark.parametrize("n,k,dist", [(1_000_000, 200, "uniform"), (1 << 22, 300_000, "zipf"),
                                      (500_000, 500_000, "uniform"), (1_000_000, 8, "uniform"),
                                      (1 << 24, 30_000, "uniform")])
def test_in_place32(ctx, n, k, dist):
    x = col32(n, k, dist=dist)
    check(ctx, x, True, label="in place", inplace=True)


@pytest.mark.parametrize("n", [3000, 100_000, 2_000_001])
def test_monotone32(ctx, n):
    """Sorted input takes MONOTONE in its own order only: keys sorted as int32
    with negatives are not sorted as uint32, and the other way round."""
    rng = np.random.default_rng(n)
    s_signed = np.sort(rng.integers(-(1 << 31), 1 << 31, size=n, dtype=np.int64).astype(np.int32))
    ro = check(ctx, s_signed.view(np.uint32), False, label="sorted int32")
    assert ro["path"] == "MONOTONE"
    ro = check(ctx, s_signed.view(np.uint32), True, label="sorted int32 as uint32")
    assert ro["path"] != "MONOTONE"
    s_unsigned = np.sort(s_signed.view(np.uint32))
    ro = check(ctx, s_unsigned, True, label="sorted uint32")
    assert ro["path"] == "MONOTONE"


def test_without_counts_or_report32(ctx):
    x = col32(700_000, 3000, dist="zipf")
    t = torch.from_numpy(x.view(np.int32).copy()).to("cuda:0")
    out, rep, uq, ct = ctx.sort(t, counts=False, report=False)
    torch.cuda.synchronize()
    assert rep is None and uq is None
    assert np.array_equal(out.cpu().numpy(), oracle.sort(x.view(np.int32), np.int32))


def key32_in_bucket(b, m, start):
    """The first 32-bit key >= start whose Eq. hash bucket at M = 2^m is b (the
    hash reads the key's zero-extended 64-bit pattern)."""
    v = start
    while ((v * PHI) & MASK64) >> (64 - m) != b:
        v += 1
    return v


def guard32(n, spill):
    """N in {8192, 8193}, stride 8: the sampled positions hold 16 keys, two in each
    of buckets 0..7 of M = 16, 64 times each (u = 16, f1 = f2 = 0, K^ = 16; Eq.
    Msize with eight keys per bucket gives M = bit_ceil(8 * 16 / 8) = 16).  Ten keys
    of bucket 10 then occur in order: k1..k8 claim the eight slots, k9 and k10 find
    the bucket full and spill ``spill`` elements between them."""
    sampled = [key32_in_bucket(b // 2, 4, 0x100 * b + 1) for b in range(16)]
    assert len(set(sampled)) == 16
    x = np.full(n, sampled[0], dtype=np.uint32)
    pos = np.arange(0, 8192, 8)
    x[pos] = np.array(sampled, dtype=np.uint32)[np.arange(1024) % 16]
    free = np.setdiff1d(np.arange(n), pos)
    ks = []
    v = 0x7000_0000
    for _ in range(10):
        v = key32_in_bucket(10, 4, v)
        ks.append(v)
        v += 1
    c9 = spill // 2
    seq = ks[:8] + [ks[8]] * c9 + [ks[9]] * (spill - c9)
    x[free[:len(seq)]] = np.array(seq, dtype=np.uint32)
    return x


@pytest.mark.parametrize("n,spill", [(8192, 4096), (8192, 4097), (8193, 4096), (8193, 4097), (8192, 5000),
                                     (8192, 2)])
@pytest.mark.parametrize("unsigned", [False, True])
def test_guard_boundary32(ctx, n, spill, unsigned):
    """Alg. 4 at eight keys per bucket: the guard fires iff 2 * spill > N."""
    x = guard32(n, spill)
    ro = check(ctx, x, unsigned, label="guard n=%d spill=%d" % (n, spill))
    assert ro["table_M"] == 16 and ro["spill_elems"] == spill and ro["k_exact"] == 26
    assert ro["path"] == ("GUARD" if 2 * spill > n else "MAIN"), ro


def test_counts_keep_32bit_width(ctx):
    """The distinct keys come back as 32-bit values: the words past K are not
    written (the uniq buffer holds exactly K int32 keys)."""
    x = col32(300_000, 5000)
    t = torch.from_numpy(x.view(np.int32).copy()).to("cuda:0")
    uq = torch.full((x.size + 8,), -7, dtype=torch.int32, device="cuda:0")
    import paper_2605_25040_amd as cafs
    out = torch.empty_like(t)
    rep = torch.zeros(cafs.report_size(), dtype=torch.uint8, device="cuda:0")
    ct = torch.empty(x.size, dtype=torch.int64, device="cuda:0")
    ws = ctx.workspace(ctx.workspace_bytes(x.size))
    rc = ctx._lib.cafs_sort_i32(ctx._h, t.data_ptr(), out.data_ptr(), x.size, uq.data_ptr(), ct.data_ptr(),
                                rep.data_ptr(), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    k = cafs.parse_report(rep)["k_exact"]
    uo, co = oracle.counts(x.view(np.int32), np.int32)
    assert k == uo.size
    assert np.array_equal(uq[:k].cpu().numpy(), uo)
    assert bool((uq[k:] == -7).all())
    assert np.array_equal(ct[:k].cpu().numpy().view(np.uint64), co)


@pytest.mark.parametrize("unsigned", [False, True])
@pytest.mark.parametrize("n,k", [(1 << 20, 1000), (300_001, 300_001), (5, 5), (2049, 3)])
def test_radix_sort_api32(ctx, n, k, unsigned):
    x = col32(n, k, dist="zipf")
    dt = np.uint32 if unsigned else np.int32
    t = torch.from_numpy(x.view(np.int32).copy()).to("cuda:0")
    y = ctx.radix_sort(t, unsigned=unsigned)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy().view(dt), oracle.sort(x.view(dt), dt))


@pytest.mark.parametrize("n,k", [(1 << 20, 1000), (4096, 8), (100_000, 100_000), (3, 3)])
def test_estimate_api32(ctx, n, k):
    """The estimate of a 32-bit column equals the oracle's estimate of the
    zero-extended keys (sampling and equality do not depend on the width)."""
    x = col32(n, k, dist="zipf")
    t = torch.from_numpy(x.view(np.int32).copy()).to("cuda:0")
    e = ctx.estimate(t)
    want = oracle.estimate(x.astype(np.uint64))
    for f in oracle.ESTIMATE_FIELDS:
        assert e[f] == want[f], (f, e, want)


def test_batched_mixed_widths(ctx):
    """One batch of int64, uint64, int32 and uint32 columns of every path."""
    import paper_2605_25040_amd as cafs
    shapes = [(100_000, 200, "uniform"), (50_000, 50_000, "uniform"), (300_000, 4, "uniform"),
              (1000, 10, "zipf"), (400_000, 20_000, "zipf"), (70_000, 300, "grouped"), (0, 1, "uniform"),
              (1 << 21, 300_000, "zipf")]
    cols, want = [], []
    dev = torch.device("cuda", 0)
    for i, (n, k, dist) in enumerate(shapes * 4):
        width, unsigned = [(8, False), (8, True), (4, False), (4, True)][i // len(shapes)]
        x64 = gen.column(n, k, dist=dist, seed=1000 + i, dtype=np.uint64)
        if width == 4:
            x = (x64 & np.uint64(0xFFFFFFFF)).astype(np.uint32)
            dt = np.uint32 if unsigned else np.int32
            t = torch.from_numpy(x.view(np.int32).copy()).to(dev)
        else:
            x = x64
            dt = np.uint64 if unsigned else np.int64
            t = torch.from_numpy(x.view(np.int64).copy()).to(dev)
        cols.append({"in": t, "out": torch.empty_like(t), "unsigned": unsigned, "uniq": torch.empty_like(t),
                     "counts": torch.empty(n, dtype=torch.int64, device=dev),
                     "report": torch.zeros(cafs.report_size(), dtype=torch.uint8, device=dev)})
        want.append((x.view(dt), dt))
    ctx.sort_batched(cols)
    torch.cuda.synchronize()
    for i, (c, (x, dt)) in enumerate(zip(cols, want)):
        r = cafs.parse_report(c["report"])
        y = c["out"].cpu().numpy().view(dt)
        assert np.array_equal(y, oracle.sort(x, dt)), "column %d" % i
        ro = oracle.report(x, dt)
        for f in oracle.REPORT_FIELDS:
            assert r[f] == ro[f], "column %d field %s gpu=%r oracle=%r" % (i, f, r[f], ro[f])
        k = r["k_exact"]
        uo, co = oracle.counts(x, dt)
        assert np.array_equal(c["uniq"][:k].cpu().numpy().view(dt), uo), "column %d" % i
        assert np.array_equal(c["counts"][:k].cpu().numpy().view(np.uint64), co), "column %d" % i


def test_noalloc_32bit(ctx):
    """The allocation-free entry point with int32 and uint32 columns, twice in a
    row with a smaller second input."""
    import paper_2605_25040_amd as cafs
    for n, k, dtc, dt in [(1 << 20, 3000, cafs.I32, np.int32), (300_000, 70_000, cafs.U32, np.uint32)]:
        x = col32(n, k, dist="zipf").view(dt)
        t = torch.from_numpy(x.view(np.int32).copy()).to("cuda:0")
        out = torch.empty_like(t)
        uq = torch.empty_like(t)
        ct = torch.empty(n, dtype=torch.int64, device="cuda:0")
        rep = torch.zeros(cafs.report_size(), dtype=torch.uint8, device="cuda:0")
        rc = ctx._lib.cafs_sort_noalloc(ctx._h, t.data_ptr(), out.data_ptr(), n, dtc, uq.data_ptr(),
                                        ct.data_ptr(), rep.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert rc == 0
        torch.cuda.synchronize()
        r = cafs.parse_report(rep)
        assert np.array_equal(out.cpu().numpy().view(dt), oracle.sort(x, dt))
        ro = oracle.report(x, dt)
        for f in oracle.REPORT_FIELDS:
            assert r[f] == ro[f], (f, r[f], ro[f])
        uo, co = oracle.counts(x, dt)
        assert np.array_equal(uq[:r["k_exact"]].cpu().numpy().view(dt), uo)
        assert np.array_equal(ct[:r["k_exact"]].cpu().numpy().view(np.uint64), co)
    assert ctypes.sizeof(cafs.Report) == cafs.report_size()
