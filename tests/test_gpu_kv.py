"""GPU parity of the key-value sort (cafs_sort_kv) against the oracle's stable
key-value sort.

Every comparison is bit-exact: the sorted keys, the payloads (each must sit at its
key's position, equal keys in input order), the distinct keys and counts, and the
report (which is the keys-only report of the same keys).  The cases reach every
way the payloads are placed: rank digits on the count paths (one to three passes,
the lookup table in LDS, in memory, or a binary search of the distinct keys when
the table would not fit), the key-value radix passes (high K, short columns, the
spill hand-over), the monotone copy and the single-key copy.
"""
import numpy as np
import pytest

import gen
import oracle
from tests import crafted

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

EINVAL = -1


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_25040_amd as cafs
    return cafs.Context(0)


def _np_dtype(kind):
    return {"i64": np.int64, "u64": np.uint64, "f64": np.float64, "i32": np.int32, "u32": np.uint32}[kind]


def _to_device(x, kind):
    if kind in ("i32", "u32"):
        return torch.from_numpy(np.ascontiguousarray(x).view(np.int32).copy()).to("cuda:0")
    if kind == "f64":
        return torch.from_numpy(np.ascontiguousarray(x).view(np.float64).copy()).to("cuda:0")
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int64).copy()).to("cuda:0")


def check_kv(ctx, x, v, kind, label=""):
    """Sort (x, v) on the GPU as `kind` keys and compare everything with the oracle."""
    import paper_2605_25040_amd as cafs
    dt = _np_dtype(kind)
    x = np.ascontiguousarray(x).view(dt)
    keys = _to_device(x, kind)
    vals = torch.from_numpy(v.view(np.int64).copy()).to("cuda:0")
    ko, vo, rep, uq, ct = ctx.sort_kv(keys, vals, unsigned=kind in ("u64", "u32"), counts=True)
    torch.cuda.synchronize()
    r = cafs.parse_report(rep)
    y = ko.cpu().numpy().view(dt)
    w = vo.cpu().numpy().view(np.uint64)
    wy, ww = oracle.sort_kv(x, v, dt)
    assert np.array_equal(y.view(np.uint8), wy.view(np.uint8)), "%s: keys differ" % label
    bad = np.flatnonzero(w != ww)
    assert bad.size == 0, "%s: %d payloads differ, first at %d" % (label, bad.size, bad[0])
    ro = oracle.report(x, dt)
    for f in oracle.REPORT_FIELDS:
        assert r[f] == ro[f], "%s: report field %s gpu=%r oracle=%r" % (label, f, r[f], ro[f])
    k = r["k_exact"]
    uo, co = oracle.counts(x, dt)
    assert np.array_equal(uq[:k].cpu().numpy().view(dt).view(np.uint8), uo.view(np.uint8)), label
    assert np.array_equal(ct[:k].cpu().numpy().view(np.uint64), co), label
    return r


def _col(n, k, dist, kind, seed=None, palette="random"):
    x = gen.column(n, k, dist=dist, s=1.1, palette=palette, seed=seed, dtype=np.uint64)
    if kind in ("i32", "u32"):
        return (x & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return x


def _payloads(n, seed, row_ids):
    if row_ids:
        return np.arange(n, dtype=np.uint64)
    return np.random.default_rng(seed).integers(0, 2**64 - 1, size=n, dtype=np.uint64, endpoint=True)


CASES = [
    # n, K, dist, expected path or None, what it reaches
    (1_000_000, 4, "uniform", "TINY"),          # rank digits, one pass, table in LDS
    (1_000_000, 1, "uniform", None),            # one key: payloads copied in order
    (1_000_000, 200, "uniform", "MAIN"),        # one pass
    (500_000, 256, "uniform", "MAIN"),          # K = 256: one pass (ranks 0..255)
    (500_000, 257, "uniform", "MAIN"),          # two passes
    (400_000, 1024, "uniform", "MAIN"),            # table of 2048 slots: the largest in LDS
    (400_000, 1100, "uniform", "MAIN"),            # table in memory
    (2_000_000, 10_000, "uniform", "MAIN"),     # pair-free ranking, two passes
    (3_000_001, 65_537, "uniform", "MAIN"),     # pair sort and three passes
    (1 << 24, 30_000, "uniform", "MAIN"),       # hash partitions
    (1 << 22, 300_000, "zipf", None),           # spill list and fold
    (100_000, 100_000, "uniform", "HIGH_K"),    # key-value radix passes
    (1000, 300, "uniform", "SMALL_N"),          # key-value radix passes (short column)
    (200_000, 300, "grouped", None),
]


@pytest.mark.parametrize("kind", ["i64", "u64", "i32"])
@pytest.mark.parametrize("n,k,dist,path", CASES)
def test_kv_paths(ctx, n, k, dist, path, kind):
    x = _col(n, k, dist, kind)
    v = _payloads(n, n + k, row_ids=(k % 2 == 0))
    r = check_kv(ctx, x, v, kind, label="%s n=%d k=%d %s" % (kind, n, k, dist))
    if path is not None:
        assert r["path"] == path, r


@pytest.mark.parametrize("kind", ["u32", "f64"])
@pytest.mark.parametrize("n,k", [(1_000_000, 8), (700_000, 3000), (100_000, 100_000), (2047, 100)])
def test_kv_other_key_types(ctx, kind, n, k):
    if kind == "f64":
        rng = np.random.default_rng(n + k)
        pal = rng.normal(size=k) * 10.0 ** rng.uniform(-30, 30, size=k)
        pal[: min(k, 4)] = np.array([0.0, -0.0, np.inf, -np.inf])[: min(k, 4)]
        x = pal[rng.integers(0, k, size=n)].view(np.uint64)
    else:
        x = _col(n, k, "zipf", kind)
    check_kv(ctx, x, _payloads(n, 3, row_ids=True), kind, label="%s n=%d k=%d" % (kind, n, k))


def test_kv_monotone_input(ctx):
    rng = np.random.default_rng(4)
    x = np.sort(rng.integers(-1000, 1000, size=300_000)).astype(np.int64).view(np.uint64)
    r = check_kv(ctx, x, _payloads(x.size, 5, row_ids=False), "i64", label="sorted")
    assert r["path"] == "MONOTONE"


@pytest.mark.parametrize("n,spill", [(8192, 4096), (8192, 4097)])
def test_kv_guard_boundary(ctx, n, spill):
    x, exp = crafted.t7_guard(n, spill)
    r = check_kv(ctx, x, _payloads(n, 6, row_ids=True), "u64", label="guard %d" % spill)
    assert r["path"] == exp["path"]


def test_kv_spill_hand_over_to_radix(ctx):
    """Keys that collide in every table overflow into the radix engine (report
    flag 1); the payloads then travel through the key-value radix passes."""
    phi = 0x9E3779B97F4A7C15
    inv = pow(phi, -1, 1 << 64)
    pal = np.array([(((0x5A5A5A5A << 32) + i) * inv) % (1 << 64) for i in range(2000)], dtype=np.uint64)
    rng = np.random.default_rng(78)
    x = pal[rng.integers(0, pal.size, size=200_000)]
    x[: pal.size] = pal
    r = check_kv(ctx, x, _payloads(x.size, 7, row_ids=True), "i64", label="overflow")
    assert r["flags"] & 1, r


def test_kv_binary_search_lookup(ctx):
    """2.5 million distinct keys on the count path (estimate 1: every sampled
    position holds one value) in a column of 2^24: the rank table would need more
    slots than the workspace's table holds, so the ranks come from a binary search
    of the distinct keys (three passes)."""
    rng = np.random.default_rng(91)
    n = 1 << 24
    stride = n // 1024
    x = np.full(n, 12345, dtype=np.uint64)
    cand = np.setdiff1d(np.arange(n), np.arange(0, n, stride))
    pos = rng.choice(cand, size=2_500_000, replace=False)
    x[pos] = rng.integers(1 << 20, 2**64, size=pos.size, dtype=np.uint64)
    r = check_kv(ctx, x, _payloads(n, 8, row_ids=True), "i64", label="binary search")
    assert r["path"] == "MAIN" and not (r["flags"] & 1) and r["k_exact"] == 2_500_001, r


@pytest.mark.parametrize("n", [0, 1, 2, 2047, 2048, 2049, 4097, 9000])
def test_kv_small_and_ragged(ctx, n):
    rng = np.random.default_rng(n + 17)
    x = rng.integers(0, max(1, n // 4 + 1), size=n).astype(np.uint64)
    check_kv(ctx, x, _payloads(n, n, row_ids=False), "i64", label="n=%d" % n)


def test_kv_full_size_properties(ctx):
    """The HBM-scale column (2^28 int64 keys, K = 1000, Zipf(1.0)) with row ids as
    payloads, checked on the GPU by the properties that fix a stable sort: the keys
    equal the keys-only sort's output, the payloads are a permutation of the row ids,
    each payload's input key is the key beside it, and within a key the row ids
    rise.  A sample of positions is checked against the oracle's counts."""
    import paper_2605_25040_amd as cafs
    n, k = 1 << 28, 1000
    x = gen.column(n, k, dist="zipf", s=1.0, palette="random", dtype=np.int64)
    keys = torch.from_numpy(x).to("cuda:0")
    del x
    vals = torch.arange(n, dtype=torch.int64, device="cuda:0")
    ko, vo, rep, _, _ = ctx.sort_kv(keys, vals)
    ref, _, _, _ = ctx.sort(keys, report=False)
    torch.cuda.synchronize()
    r = cafs.parse_report(rep)
    assert r["path"] == "MAIN" and r["k_exact"] == k
    assert torch.equal(ko, ref)
    del ref, vals
    seen = torch.zeros(n, dtype=torch.int8, device="cuda:0")
    seen.index_fill_(0, vo, 1)
    assert bool(seen.all()), "payloads are not a permutation of the row ids"
    del seen
    assert torch.equal(keys[vo], ko), "a payload sits beside another key"
    same = ko[1:] == ko[:-1]
    assert bool((vo[1:][same] > vo[:-1][same]).all()), "row ids of one key out of input order"
    torch.cuda.empty_cache()


def test_kv_errors(ctx):
    n = 10_000
    buf = torch.zeros(4 * n, dtype=torch.int64, device="cuda:0")
    buf[:n] = torch.arange(n, 0, -1, device="cuda:0")
    p = buf.data_ptr()
    ws = ctx.workspace(ctx.workspace_bytes(n))
    s = torch.cuda.current_stream().cuda_stream
    lib = ctx._lib

    def call(kin, kout, vin, vout, dtype=0, nn=n):
        return lib.cafs_sort_kv(ctx._h, kin, kout, vin, vout, nn, dtype, None, None, None, ws.data_ptr(),
                                ws.numel(), s)
    K_IN, K_OUT, V_IN, V_OUT = p, p + n * 8, p + 2 * n * 8, p + 3 * n * 8
    assert call(K_IN, K_IN, V_IN, V_OUT) == EINVAL                # keys in place
    assert call(K_IN, K_OUT, V_IN, V_IN) == EINVAL                # payloads in place
    assert call(K_IN, K_OUT, V_IN, K_OUT + 8) == EINVAL           # payload output over the key output
    assert call(K_IN, V_IN - 8, V_IN, V_OUT) == EINVAL            # key output over the payload input
    assert call(K_IN, K_OUT, None, V_OUT) == EINVAL
    assert call(K_IN, K_OUT, V_IN + 4, V_OUT) == EINVAL           # misaligned payloads
    assert call(K_IN, K_OUT, V_IN, V_OUT, dtype=9) == EINVAL
    torch.cuda.synchronize()
    assert bool((buf[n:] == 0).all()), "a rejected call wrote memory"
    assert call(K_IN, K_OUT, V_IN, V_OUT) == 0
    torch.cuda.synchronize()
    assert torch.equal(buf[n:2 * n], torch.arange(1, n + 1, device="cuda:0"))
