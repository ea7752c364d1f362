"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer work, so every comparison is bit-exact: the sorted output, the distinct
keys and their counts, and every report field (estimate, path, tiny miss, M,
spill, K).  Inputs are seeded synthetic columns (gen/) and the hand-built
dispatcher / guard cases (tests/crafted.py).
"""
import numpy as np
import pytest

import gen
import oracle
from tests import crafted

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_25040_amd as cafs
    return cafs.Context(0)


ORACLE_FIELDS = oracle.REPORT_FIELDS


def run_gpu(ctx, x_np, unsigned, counts=True, shift_in=0, shift_out=0, inplace=False):
    """Sort x_np on the GPU; optional 8-byte misalignment of input/output."""
    import paper_2605_25040_amd as cafs
    n = x_np.size
    xi = x_np.view(np.int64)
    buf = torch.empty(n + 2, dtype=torch.int64, device="cuda:0")
    buf[shift_in:shift_in + n].copy_(torch.from_numpy(xi.copy()))
    x = buf[shift_in:shift_in + n]
    if inplace:
        out = x
    else:
        obuf = torch.empty(n + 2, dtype=torch.int64, device="cuda:0")
        out = obuf[shift_out:shift_out + n]
    out, rep, uq, ct = ctx.sort(x, unsigned=unsigned, out=out, counts=counts)
    torch.cuda.synchronize()
    r = cafs.parse_report(rep)
    y = out.cpu().numpy().view(np.uint64 if unsigned else np.int64)
    if counts:
        k = r["k_exact"]
        u = uq[:k].cpu().numpy().view(np.uint64 if unsigned else np.int64)
        c = ct[:k].cpu().numpy().view(np.uint64)
    else:
        u = c = None
    return y, r, u, c


def check(ctx, x_np, unsigned, label="", **kw):
    dt = np.uint64 if unsigned else np.int64
    x = x_np.view(dt)
    y, r, u, c = run_gpu(ctx, x_np, unsigned, **kw)
    want = oracle.sort(x, dt)
    assert np.array_equal(y, want), "%s: sorted output differs" % label
    ro = oracle.report(x, dt)
    for f in ORACLE_FIELDS:
        assert r[f] == ro[f], "%s: report field %s gpu=%r oracle=%r (gpu %r)" % (label, f, r[f], ro[f], r)
    if u is not None:
        uo, co = oracle.counts(x, dt)
        assert np.array_equal(u, uo), "%s: distinct keys differ" % label
        assert np.array_equal(c, co), "%s: counts differ" % label
    return r


SEEDED = [
    # n, K, dist, s, palette
    (3000, 5, "uniform", 1.1, "random"),
    (5000, 200, "uniform", 1.1, "random"),
    (131_072 + 123, 200, "uniform", 1.1, "random"),
    (200_000, 1000, "zipf", 1.0, "random"),
    (250_000, 3000, "zipf", 1.1, "random"),
    (300_001, 10_000, "uniform", 1.1, "random"),   # K > 8192: pair sort
    (100_000, 100_000, "uniform", 1.1, "random"),  # all distinct: HIGH_K
    (1_000_000, 200, "uniform", 1.1, "random"),    # the plain single-column config
    (1_000_000, 4, "uniform", 1.1, "random"),      # tiny
    (1_000_000, 8, "zipf", 1.1, "random"),         # tiny
    (400_000, 1000, "uniform", 1.1, "codes"),      # dictionary codes 0..K-1
    (200_000, 64, "runs", 1.1, "random"),
    (200_000, 300, "grouped", 1.1, "random"),      # sorted by group -> MONOTONE
    (200_000, 300, "almost_sorted", 1.1, "ap"),
    (60_000, 30_000, "zipf", 1.1, "random"),       # Chao1 underestimate
    (2_000_000, 200_000, "zipf", 1.1, "random"),   # underestimate: table overflow -> radix engine
    (500_000, 150_000, "uniform", 1.1, "random"),
    # every workgroup sees most keys: full LDS windows, deferred second pass
    (1 << 24, 12_000, "uniform", 1.1, "random"),
    (1 << 23, 10_000, "zipf", 1.1, "random"),
    (1 << 23, 20_000, "uniform", 1.1, "random"),     # beyond the LDS table: deferred pass overflows to global
    (3_000_001, 100_000, "uniform", 1.1, "random"),  # deferral regions fill up
    # estimates on both sides of the LDS bucket width switch (2 keys below 1800, 4 above)
    (2_000_000, 1_700, "uniform", 1.1, "random"),
    (2_000_000, 1_900, "uniform", 1.1, "random"),
    (1 << 23, 20_000, "zipf", 1.1, "random"),        # estimate ~2200 for 20000 keys: table far past capacity
    # hash partitions of the count workgroups (2, 8 and 16 partitions)
    (1 << 24, 10_000, "uniform", 1.1, "random"),
    (1 << 24, 30_000, "uniform", 1.1, "random"),
    (1 << 24, 100_000, "uniform", 1.1, "codes"),
    (1_500_001, 150_000, "uniform", 1.1, "random"),
    # heavy tails far past the estimate: keys beyond the global table's limit spill
    (1 << 22, 300_000, "zipf", 1.1, "random"),
    (1 << 22, 1_000_000, "zipf", 1.1, "random"),
    (3_000_000, 3_000_000, "zipf", 1.1, "random"),
]


@pytest.mark.parametrize("unsigned", [False, True])
@pytest.mark.parametrize("n,k,dist,s,pal", SEEDED)
def test_seeded_columns(ctx, n, k, dist, s, pal, unsigned):
    x = gen.column(n, k, dist=dist, s=s, palette=pal, dtype=np.uint64)
    check(ctx, x, unsigned, label="%s n=%d k=%d" % (dist, n, k))


@pytest.mark.parametrize("name", list(crafted.all_cases().keys()))
@pytest.mark.parametrize("unsigned", [False, True])
def test_crafted(ctx, name, unsigned):
    x, exp = crafted.all_cases()[name]
    r = check(ctx, x, unsigned, label=name)
    for key, val in exp.items():
        assert r[key] == val, (name, key, r[key], val)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 64, 2047, 2048, 2049, 4095, 4097, 8193, 9000])
@pytest.mark.parametrize("unsigned", [False, True])
def test_small_and_ragged(ctx, n, unsigned):
    x = gen.column(n, max(1, n // 3), dtype=np.uint64)
    check(ctx, x, unsigned, label="n=%d" % n)


@pytest.mark.parametrize("n", [0, 1, 2047, 2048, 100_000])
def test_sorted_inputs(ctx, n):
    x, _ = crafted.t1_sorted(n)
    r = check(ctx, x, False, label="sorted n=%d" % n)
    assert r["path"] == "MONOTONE"


def test_extreme_values_every_path(ctx):
    ext = np.array([0, 1, (1 << 63) - 1, 1 << 63, (1 << 64) - 1, (1 << 64) - 2, 5, 1 << 62],
                   dtype=np.uint64)
    rng = np.random.default_rng(10)
    for n, kk in ((1000, 8), (50_000, 3), (50_000, 8), (80_000, 1000)):
        pal = np.concatenate([ext, rng.integers(0, 2**63, size=max(0, kk - ext.size), dtype=np.uint64)])[:max(kk, 3)]
        x = pal[rng.integers(0, pal.size, size=n)]
        for unsigned in (False, True):
            check(ctx, x, unsigned, label="extremes n=%d k=%d" % (n, kk))


@pytest.mark.parametrize("shift_in,shift_out", [(1, 0), (0, 1), (1, 1)])
def test_misaligned_buffers(ctx, shift_in, shift_out):
    for n, k in ((100_001, 50), (100_001, 4), (20_001, 20_001)):
        x = gen.column(n, k, dtype=np.uint64)
        check(ctx, x, False, label="misaligned n=%d k=%d" % (n, k), shift_in=shift_in, shift_out=shift_out)


def test_in_place(ctx):
    for n, k, dist in ((300_000, 200, "uniform"), (5000, 5000, "uniform"), (100_000, 4, "uniform"),
                       (100_000, 300, "grouped"),
                       (300_001, 10_000, "uniform"),      # pair sort, guard with contested buckets
                       (2_000_000, 200_000, "zipf"),      # table overflow: radix engine on the main path
                       (60_000, 30_000, "zipf")):
        x = gen.column(n, k, dist=dist, dtype=np.uint64)
        check(ctx, x, False, label="inplace n=%d k=%d" % (n, k), inplace=True)
    for name in ("t7_even_fire", "t8_big_last", "t9_tiny_miss_guard"):
        x, _ = crafted.all_cases()[name]
        check(ctx, x, False, label="inplace " + name, inplace=True)


def test_without_counts_or_report(ctx):
    x = gen.column(300_000, 700, dist="zipf", s=1.0, dtype=np.uint64)
    xt = torch.from_numpy(x.view(np.int64).copy()).cuda()
    out, rep, uq, ct = ctx.sort(xt, report=False)
    torch.cuda.synchronize()
    assert rep is None
    assert np.array_equal(out.cpu().numpy(), oracle.sort(x.view(np.int64)))


def test_estimate_api(ctx):
    for n, k, dist in ((0, 1, "uniform"), (5, 5, "uniform"), (5000, 200, "uniform"),
                       (1_000_000, 1000, "zipf"), (100_000, 100_000, "uniform")):
        x = gen.column(n, k, dist=dist, dtype=np.uint64)
        e = ctx.estimate(torch.from_numpy(x.view(np.int64).copy()).cuda())
        assert e == oracle.estimate(x), (n, k, dist)


@pytest.mark.parametrize("unsigned", [False, True])
def test_radix_sort_api(ctx, unsigned):
    for n, k, pal in ((1, 1, "random"), (4095, 4095, "random"), (300_000, 300_000, "random"),
                      (200_000, 1000, "codes"), (100_003, 3, "random")):
        x = gen.column(n, k, palette=pal, dtype=np.uint64)
        xt = torch.from_numpy(x.view(np.int64).copy()).cuda()
        y = ctx.radix_sort(xt, unsigned=unsigned)
        torch.cuda.synchronize()
        dt = np.uint64 if unsigned else np.int64
        assert np.array_equal(y.cpu().numpy().view(dt), np.sort(x.view(dt)))


def test_deterministic_reports(ctx):
    x = gen.column(500_000, 2000, dist="zipf", s=1.1, dtype=np.uint64)
    a = run_gpu(ctx, x, False)
    b = run_gpu(ctx, x, False)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


@pytest.mark.parametrize("k", [8191, 8192, 8193, 32767, 32768, 32769])
@pytest.mark.parametrize("with_marker", [False, True])
def test_order_boundaries(ctx, k, with_marker):
    """K at the edges of the rank order (K <= 32768) and the pair radix sort above,
    with and without the empty-slot marker value among the keys."""
    rng = np.random.default_rng(k)
    pal = np.unique(rng.integers(0, 2**64 - 2, size=k + 64, dtype=np.uint64))[:k]
    if with_marker:
        pal[0] = np.uint64(2**64 - 1)
    n = 40 * k
    x = np.concatenate([pal, pal[rng.integers(0, k, size=n - k)]])
    rng.shuffle(x)
    for unsigned in (False, True):
        r = check(ctx, x, unsigned, label="order k=%d marker=%s" % (k, with_marker))
        assert r["k_exact"] == k


@pytest.mark.gpu
@pytest.mark.parametrize("n,k", [(300_001, 1000), (300_001, 5000), (400_001, 40_000)])
def test_head_pair_single_first_run(ctx, n, k):
    """Output 8 bytes off 16-byte alignment, so that the first output pair holds only
    element 0, and the smallest key occurring exactly once (a first run of length
    one): row emit (K <= 32768) and the pair-sort emit (K above it)."""
    rng = np.random.default_rng(n + k)
    pal = np.unique(rng.integers(1, 2**62, size=k + 64, dtype=np.int64))[:k]
    rest = pal[1:][rng.integers(0, k - 1, size=n - 1)]
    rest[: k - 1] = pal[1:]  # every key present
    x = np.concatenate([pal[:1], rest])
    rng.shuffle(x)
    for shift_out in (1, 0):
        r = check(ctx, x.view(np.uint64), False, label="head n=%d k=%d shift=%d" % (n, k, shift_out),
                  shift_out=shift_out)
        assert r["k_exact"] == k and r["path"] == "MAIN"


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1_000_000, 1_000_001])
def test_emit_crowded_segment(ctx, n):
    """One key holds 90% of the column and sorts first; 29999 keys share the rest, so
    the last segments of the row emit hold thousands of runs each (more than one
    workgroup stages) and search the global run offsets."""
    rng = np.random.default_rng(n)
    k = 30_000
    pal = np.unique(rng.integers(1, 2**62, size=k + 64, dtype=np.int64))[:k - 1]
    m = n // 10
    rest = pal[rng.integers(0, k - 1, size=m)]
    rest[: k - 1] = pal
    x = np.concatenate([np.full(n - m, -7, dtype=np.int64), rest])
    rng.shuffle(x)
    for shift_out in (0, 1):
        r = check(ctx, x.view(np.uint64), False, label="crowded n=%d shift=%d" % (n, shift_out),
                  shift_out=shift_out)
        assert r["k_exact"] == k and r["path"] == "MAIN" and r["engine"] == "HASH"


def _colliding_keys(k):
    """k distinct keys whose products with the multiplier of Eq. hash share their top
    32 bits (y * phi^-1 mod 2^64 for y with equal high words): one bucket of every
    table hashed with that multiplier."""
    phi = 0x9E3779B97F4A7C15
    inv = pow(phi, -1, 1 << 64)
    top = 0x5A5A5A5A << 32
    return np.array([((top + i) * inv) % (1 << 64) for i in range(k)], dtype=np.uint64)


@pytest.mark.gpu
def test_hash_seed(ctx):
    """Seeded count tables: outputs, counts and reports equal the oracle's for any
    seed; keys that all collide under the paper's multiplier overflow the tables
    without a seed and stay on the hash count with one."""
    rng = np.random.default_rng(77)
    pal = _colliding_keys(2000)
    x_col = pal[rng.integers(0, pal.size, size=1_000_000)]
    x_col[: pal.size] = pal
    cols = [gen.column(1_000_000, 1000, dist="zipf", s=1.0, palette="random", dtype=np.uint64),
            gen.column(1 << 22, 12_000, dist="uniform", palette="random", dtype=np.uint64),
            gen.column(2_000_000, 200_000, dist="zipf", s=1.1, palette="random", dtype=np.uint64)]
    try:
        r0 = check(ctx, x_col, True, label="colliding, default multiplier")
        assert r0["flags"] & 1, "colliding keys were expected to overflow the fixed-multiplier tables"
        for seed in (1, 2**63 + 5, 123456789):
            ctx.set_hash_seed(seed)
            r = check(ctx, x_col, True, label="colliding, seed %d" % seed)
            assert r["engine"] == "HASH" and not (r["flags"] & 1), r
            for i, x in enumerate(cols):
                check(ctx, x, False, label="seed %d column %d" % (seed, i))
    finally:
        ctx.set_hash_seed(0)


# ---- float64 keys (IEEE 754 totalOrder) --------------------------------------

def _f64_column(n, k, dist, seed, specials=False):
    """n doubles from a palette of k values (normal times a power of ten, optionally
    with signed zeros, infinities, subnormals and NaNs of both signs), drawn with
    the generator's frequency model over dictionary codes."""
    rng = np.random.default_rng(seed)
    pal = rng.normal(size=k) * 10.0 ** rng.uniform(-30, 30, size=k)
    if specials and k >= 12:
        sp = np.array([0x0, 0x8000000000000000, 0x7FF0000000000000, 0xFFF0000000000000, 0x1, 0x8000000000000001,
                       0x7FF8000000000000, 0xFFF8000000000000, 0x7FF8000000000005], dtype=np.uint64)
        pal[:sp.size] = sp.view(np.float64)
    pal = np.unique(pal.view(np.uint64)).view(np.float64)  # distinct bit patterns
    codes = gen.column(n, pal.size, dist=dist, s=1.1, palette="codes", seed=seed, dtype=np.uint64)
    return pal[codes.astype(np.int64)]


def check_f64(ctx, x, label):
    import paper_2605_25040_amd as cafs
    xt = torch.from_numpy(x.copy()).to("cuda:0")
    out, rep, uq, ct = ctx.sort(xt, counts=True)
    torch.cuda.synchronize()
    r = cafs.parse_report(rep)
    y = out.cpu().numpy()
    want = oracle.sort(x, np.float64)
    assert np.array_equal(y.view(np.uint64), want.view(np.uint64)), "%s: sorted output differs" % label
    ro = oracle.report(x, np.float64)
    for f in ORACLE_FIELDS:
        assert r[f] == ro[f], "%s: report field %s gpu=%r oracle=%r" % (label, f, r[f], ro[f])
    k = r["k_exact"]
    uo, co = oracle.counts(x, np.float64)
    assert np.array_equal(uq[:k].cpu().numpy().view(np.uint64), uo.view(np.uint64)), "%s: distinct keys" % label
    assert np.array_equal(ct[:k].cpu().numpy().view(np.uint64), co), "%s: counts" % label
    return r


F64_CASES = [
    # n, k, dist, specials: every dispatcher path and both engines
    (1500, 40, "uniform", True),          # N < 2048: radix engine
    (300_000, 5, "uniform", False),       # tiny
    (400_000, 12, "zipf", True),          # tiny check misses an unsampled NaN or zero: main path
    (1_000_000, 300, "zipf", True),       # main path, ranking
    (2_000_000, 3000, "uniform", True),   # 4-key LDS buckets
    (600_000, 20_000, "uniform", True),   # pair sort (K above the ranking limit)
    (2_000_000, 200_000, "zipf", True),   # table overflow: radix engine, general guard
    (200_000, 150_000, "uniform", True),  # high K
]


@pytest.mark.parametrize("n,k,dist,specials", F64_CASES)
def test_f64_columns(ctx, n, k, dist, specials):
    x = _f64_column(n, k, dist, seed=n + k, specials=specials)
    check_f64(ctx, x, "f64 n=%d k=%d %s" % (n, k, dist))


def test_f64_monotone_and_radix_api(ctx):
    x = np.sort(_f64_column(300_000, 500, "uniform", seed=9, specials=True))
    x = oracle.sort(x, np.float64)  # totalOrder, which places -0, +0 and NaNs by bits
    r = check_f64(ctx, x, "f64 sorted")
    assert r["path"] == "MONOTONE"
    y = _f64_column(1_000_003, 70_000, "zipf", seed=10, specials=True)
    out = ctx.radix_sort(torch.from_numpy(y.copy()).to("cuda:0"))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), oracle.sort(y, np.float64).view(np.uint64))


# ---- run-length injection (structured inputs) --------------------------------

RLE_CASES = [
    # n, K, dist: runs of mean length n / (4K) ("runs"), sorted-by-group runs of
    # n / K ("grouped", random palette: not monotone), 1% swaps of those ("almost_sorted")
    (1 << 22, 64, "runs"),           # runs of ~16k: whole slices merge
    (1 << 22, 10_000, "runs"),       # runs of ~100: cut at slice ends
    (1 << 22, 300_000, "runs"),      # runs of 1-6: mostly below the merge threshold
    (1 << 23, 20_000, "runs"),       # beyond the LDS table: deferred heads carry their runs
    (1 << 22, 1000, "grouped"),
    (3_000_001, 5000, "almost_sorted"),
    (1 << 22, 7, "runs"),            # tiny path
]


@pytest.mark.parametrize("n,k,dist", RLE_CASES)
def test_run_length_inputs(ctx, n, k, dist):
    x = gen.column(n, k, dist=dist, s=1.1, palette="random", dtype=np.uint64)
    check(ctx, x, True, label="%s n=%d k=%d" % (dist, n, k))
    check(ctx, x, False, label="%s n=%d k=%d signed" % (dist, n, k))


def test_runs_of_every_length_across_slices(ctx):
    """Runs of lengths 1..300 in a shuffled order, so that heads fall at every
    position of a wave's 128-element slice, next to single elements."""
    rng = np.random.default_rng(21)
    lens = np.concatenate([np.arange(1, 301), rng.integers(1, 300, size=6000)])
    rng.shuffle(lens)
    vals = rng.integers(0, 2**63, size=500, dtype=np.int64).view(np.uint64)
    keys = vals[rng.integers(0, vals.size, size=lens.size)]
    x = np.repeat(keys, lens)
    check(ctx, x, True, label="mixed runs")
    check(ctx, x[::-1].copy(), False, label="mixed runs reversed")


# ---- HIP graph capture ---------------------------------------------------------

def test_graph_capture_replays(ctx):
    """A captured call replays correctly: other columns (other dispatcher paths and
    engines) are copied into the captured input buffer between replays, with eager
    calls and synchronisations in between, and every replay is checked against the
    oracle."""
    import paper_2605_25040_amd as cafs
    n = 1_000_003
    shapes = ((1000, "zipf"), (5, "uniform"), (20_000, "uniform"), (300_000, "uniform"), (64, "runs"))
    cols = [gen.column(n, k, dist=d, s=1.1, palette="random", dtype=np.uint64) for k, d in shapes]
    x = torch.empty(n, dtype=torch.int64, device="cuda:0")
    out = torch.empty_like(x)
    ws = ctx.workspace(ctx.workspace_bytes(n))
    x.copy_(torch.from_numpy(cols[0].view(np.int64).copy()))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.sort(x, unsigned=True, out=out, counts=True, ws=ws)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            res = ctx.sort(x, unsigned=True, out=out, counts=True, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    _, rep_g, uq_g, ct_g = res
    for rnd in range(2):
        for (k, d), c in zip(shapes, cols):
            label = "replay %d %s k=%d" % (rnd, d, k)
            x.copy_(torch.from_numpy(c.view(np.int64).copy()))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint64), oracle.sort(c, np.uint64)), label
            r = cafs.parse_report(rep_g)
            ro = oracle.report(c, np.uint64)
            for f in ORACLE_FIELDS:
                assert r[f] == ro[f], (label, f, r[f], ro[f])
            uo, co = oracle.counts(c, np.uint64)
            kk = r["k_exact"]
            assert np.array_equal(uq_g[:kk].cpu().numpy().view(np.uint64), uo), label
            assert np.array_equal(ct_g[:kk].cpu().numpy().view(np.uint64), co), label
            # eager work on the same workspace between replays
            y, _, _, _ = ctx.sort(x, unsigned=True, ws=ws)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy().view(np.uint64), oracle.sort(c, np.uint64)), label + " eager"


def test_empty_marker_pattern_in_every_shape(ctx):
    """The all-ones pattern (the count tables' empty-slot marker, a negative NaN as
    float64, -1 as int64) mixed with extreme patterns, as float64 on every path and
    in long runs (the run-length path skips slices that hold it)."""
    ext = np.array([0xFFFFFFFFFFFFFFFF, 0x7FFFFFFFFFFFFFFF, 0x8000000000000000, 0x0, 0xFFF0000000000000,
                    0x7FF0000000000000, 0x1, 0xFFFFFFFFFFFFFFFE], dtype=np.uint64)
    rng = np.random.default_rng(44)
    for n, kk in ((1000, 8), (50_000, 3), (50_000, 8), (80_000, 1000), (1_000_000, 5000)):
        extra = (rng.normal(size=max(0, kk - ext.size)) * 1e6).view(np.uint64)
        pal = np.concatenate([ext, extra])[:max(kk, 3)]
        x = pal[rng.integers(0, pal.size, size=n)]
        check_f64(ctx, x.view(np.float64), "f64 extremes n=%d k=%d" % (n, kk))
    lens = rng.integers(1, 5000, size=400)
    keys = ext[rng.integers(0, ext.size, size=lens.size)]
    x = np.repeat(keys, lens)
    check_f64(ctx, x.view(np.float64), "f64 runs of extremes")
    check(ctx, x, False, label="i64 runs of extremes")
    check(ctx, x, True, label="u64 runs of extremes")


def test_spill_list_then_fold(ctx):
    """A column of 2^18 keys whose estimate is 1 (every sampled position, and most
    others, hold one value) with 80000 distinct values elsewhere: more keys than the
    global table has slots (2^16), so at least 14464 of them spill (at most 47232,
    below the radix hand-over at n / 4), and the spill list is sorted and folded with
    the table's pairs (report flag 4).  (The paper's table has M = 8 buckets; its
    spill, about 80000 elements, stays below n / 2, so the path is MAIN.)"""
    rng = np.random.default_rng(77)
    n = 1 << 18
    stride = n // 1024
    x = np.full(n, 12345, dtype=np.uint64)
    pos = rng.choice(np.setdiff1d(np.arange(n), np.arange(0, n, stride)), size=80_000, replace=False)
    x[pos] = rng.integers(1 << 20, 2**64, size=pos.size, dtype=np.uint64)
    for unsigned in (False, True):
        r = check(ctx, x, unsigned, label="spill")
        assert r["engine"] == "HASH" and r["flags"] & 4 and not r["flags"] & 1, r
        assert r["path"] == "MAIN" and r["tiny_miss"] == 1, r
    # the same in place
    y, r, _, _ = run_gpu(ctx, x, False, inplace=True)
    assert np.array_equal(y, oracle.sort(x.view(np.int64), np.int64)) and r["flags"] & 4


def test_spill_past_quarter_goes_to_radix(ctx):
    """2000 keys built to share one slot of every table hashed with the paper's
    multiplier: they overfill the LDS buckets and the global table's probe window,
    so their elements spill one by one; past n / 4 spilled pairs the radix engine
    sorts the column instead (report flag 1)."""
    rng = np.random.default_rng(78)
    pal = _colliding_keys(2000)
    x = pal[rng.integers(0, pal.size, size=200_000)]
    x[: pal.size] = pal
    r = check(ctx, x, False, label="spill overflow")
    assert r["flags"] & 1, r  # (the engine field keeps the plan's engine; flag 1 names the hand-over)


@pytest.mark.parametrize("n,k,dist", [(1 << 22, 300_000, "zipf"), (1 << 24, 30_000, "uniform")])
def test_spill_and_partitions_in_place_and_misaligned(ctx, n, k, dist):
    x = gen.column(n, k, dist=dist, s=1.1, dtype=np.uint64)
    check(ctx, x, False, label="in place", inplace=True)
    check(ctx, x, True, label="misaligned", shift_in=1, shift_out=1)
