"""Batched sorting (one launch sequence for many columns) against the oracle and
against the single-column call on the same column: bit-identical outputs,
counts and reports."""
import numpy as np
import pytest

import gen
import oracle
from tests import crafted
from tests.test_gpu_parity import check as check_single

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_25040_amd as cafs
    return cafs.Context(0)


def make_cols(arrays, unsigned_flags, counts_flags, report_flags, inplace_flags=None, shift_flags=None):
    import paper_2605_25040_amd as cafs
    cols = []
    for i, x in enumerate(arrays):
        n = x.size
        sh = shift_flags[i] if shift_flags else 0
        buf = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
        if n:
            buf[sh:sh + n].copy_(torch.from_numpy(x.view(np.int64).copy()))
        xin = buf[sh:sh + n]
        out = xin if (inplace_flags and inplace_flags[i]) else torch.empty(n, dtype=torch.int64, device="cuda:0")
        want_counts = counts_flags[i]
        cols.append(dict(
            **{"in": xin}, out=out, unsigned=unsigned_flags[i],
            uniq=torch.empty(max(n, 1), dtype=torch.int64, device="cuda:0") if want_counts else None,
            counts=torch.empty(max(n, 1), dtype=torch.int64, device="cuda:0") if want_counts else None,
            report=torch.zeros(cafs.report_size(), dtype=torch.uint8, device="cuda:0")
            if (report_flags[i] or want_counts) else None,
            src=x))
    return cols


def check_cols(cols, label):
    import paper_2605_25040_amd as cafs
    torch.cuda.synchronize()
    for i, c in enumerate(cols):
        dt = np.uint64 if c["unsigned"] else np.int64
        x = c["src"].view(dt)
        y = c["out"].cpu().numpy().view(dt)
        want = oracle.sort(x, dt)
        if not np.array_equal(y, want):
            # what the column took on the GPU, and where the output first differs
            r = cafs.parse_report(c["report"]) if c["report"] is not None else None
            bad = np.flatnonzero(y != want) if y.size == want.size else np.array([-1])
            raise AssertionError("%s col %d output: n=%d, report %r, first difference at %d of %d differing" %
                                 (label, i, x.size, r, int(bad[0]), bad.size))
        if c["report"] is not None:
            r = cafs.parse_report(c["report"])
            ro = oracle.report(x, dt)
            for f in oracle.REPORT_FIELDS:
                assert r[f] == ro[f], "%s col %d field %s gpu=%r oracle=%r" % (label, i, f, r[f], ro[f])
            if c["uniq"] is not None:
                k = r["k_exact"]
                uo, co = oracle.counts(x, dt)
                assert np.array_equal(c["uniq"][:k].cpu().numpy().view(dt), uo), (label, i)
                assert np.array_equal(c["counts"][:k].cpu().numpy().view(np.uint64), co), (label, i)


def test_batch_mixed_shapes(ctx):
    spec = gen.batch_spec(160, seed=3, n_lo=10, n_hi=3e5, k_cap=3e4)
    arrays = [gen.column(c["n"], c["k"], dist=c["dist"], s=c["s"], seed=c["seed"], dtype=np.uint64) for c in spec]
    arrays += [np.zeros(0, dtype=np.uint64), np.array([5], dtype=np.uint64),
               crafted.t1_sorted(50_000)[0]]
    m = len(arrays)
    rng = np.random.default_rng(5)
    cols = make_cols(arrays, unsigned_flags=list(rng.random(m) < 0.3), counts_flags=list(rng.random(m) < 0.5),
                     report_flags=list(rng.random(m) < 0.8), inplace_flags=list(rng.random(m) < 0.2),
                     shift_flags=[int(v) for v in rng.integers(0, 2, size=m)])
    ctx.sort_batched(cols)
    check_cols(cols, "mixed")


def test_batch_crafted_cases(ctx):
    cases = crafted.all_cases()
    arrays = [x for x, _ in cases.values()]
    m = len(arrays)
    cols = make_cols(arrays, [False] * m, [True] * m, [True] * m)
    ctx.sort_batched(cols)
    check_cols(cols, "crafted")
    import paper_2605_25040_amd as cafs
    for (name, (_, exp)), c in zip(cases.items(), cols):
        r = cafs.parse_report(c["report"])
        for k, v in exp.items():
            assert r[k] == v, (name, k, r[k], v)


def test_batch_equals_single_calls(ctx):
    """Alone and in the mix: each column's output and report are bit-identical."""
    import paper_2605_25040_amd as cafs
    spec = gen.batch_spec(600, seed=11, n_lo=1e3, n_hi=1e7, total=1 << 23)
    arrays = [gen.column(c["n"], c["k"], dist=c["dist"], s=c["s"], seed=c["seed"], dtype=np.uint64) for c in spec]
    m = len(arrays)
    cols = make_cols(arrays, [False] * m, [False] * m, [True] * m)
    ctx.sort_batched(cols)
    torch.cuda.synchronize()
    for i in range(0, m, 7):
        c = cols[i]
        out, rep, _, _ = ctx.sort(c["in"].clone())
        torch.cuda.synchronize()
        assert torch.equal(out, c["out"]), i
        ra, rb = cafs.parse_report(rep), cafs.parse_report(c["report"])
        # (engine and flags tell what ran; a spill of a few keys can depend on timing)
        assert all(ra[f] == rb[f] for f in oracle.REPORT_FIELDS), (i, ra, rb)
    # oracle on a sample of columns
    sub = [cols[i] for i in range(0, m, 29)]
    check_cols(sub, "sample")


def test_batch_hash_seed(ctx):
    """A seeded context hashes every column of a batch with its multiplier: keys
    that all collide under Eq. hash stay on the hash count, and the outputs,
    counts and reports equal the oracle's."""
    import paper_2605_25040_amd as cafs
    phi = 0x9E3779B97F4A7C15
    inv = pow(phi, -1, 1 << 64)
    pal = np.array([(((0x3C3C3C3C << 32) + i) * inv) % (1 << 64) for i in range(1500)], dtype=np.uint64)
    rng = np.random.default_rng(8)
    arrays = []
    for n in (400_000, 90_000, 700_001):
        x = pal[rng.integers(0, pal.size, size=n)]
        x[: pal.size] = pal
        arrays.append(x)
    spec = gen.batch_spec(40, seed=21, n_lo=1e3, n_hi=3e5, k_cap=3e4)
    arrays += [gen.column(c["n"], c["k"], dist=c["dist"], s=c["s"], seed=c["seed"], dtype=np.uint64) for c in spec]
    m = len(arrays)
    try:
        ctx.set_hash_seed(99)
        cols = make_cols(arrays, [True] * m, [True] * m, [True] * m)
        ctx.sort_batched(cols)
        check_cols(cols, "seeded")
        for c in cols[:3]:
            r = cafs.parse_report(c["report"])
            assert r["engine"] == "HASH" and not (r["flags"] & 1), r
    finally:
        ctx.set_hash_seed(0)


def test_batch_f64_columns(ctx):
    """float64 columns (totalOrder) mixed with int64 and uint64 ones in one batch."""
    rng = np.random.default_rng(12)
    arrays, kinds = [], []
    for i in range(24):
        n = int(rng.integers(1000, 300_000)); k = int(rng.integers(2, max(3, n // 4)))
        pal = rng.normal(size=k) * 10.0 ** rng.uniform(-8, 8, size=k)
        pal[: min(k, 3)] = np.array([0x0, 0x8000000000000000, 0x7FF8000000000000], dtype=np.uint64)[: min(k, 3)].view(np.float64)
        arrays.append(pal[rng.integers(0, k, size=n)]); kinds.append("f")
    spec = gen.batch_spec(16, seed=4, n_lo=1e3, n_hi=2e5, k_cap=2e4)
    for c in spec:
        arrays.append(gen.column(c["n"], c["k"], dist=c["dist"], s=c["s"], seed=c["seed"], dtype=np.uint64)); kinds.append("u")
    cols = []
    import paper_2605_25040_amd as cafs
    for x, kd in zip(arrays, kinds):
        n = x.size
        t = torch.from_numpy(x.copy()).to("cuda:0") if kd == "f" else torch.from_numpy(x.view(np.int64).copy()).to("cuda:0")
        cols.append(dict(**{"in": t}, out=torch.empty_like(t), unsigned=(kd == "u"),
                         uniq=torch.empty_like(t), counts=torch.empty(n, dtype=torch.int64, device="cuda:0"),
                         report=torch.zeros(cafs.report_size(), dtype=torch.uint8, device="cuda:0"), src=x, kind=kd))
    ctx.sort_batched(cols)
    torch.cuda.synchronize()
    for i, c in enumerate(cols):
        dt = np.float64 if c["kind"] == "f" else np.uint64
        x = c["src"].view(dt)
        y = c["out"].cpu().numpy().view(np.uint64)
        assert np.array_equal(y, oracle.sort(x, dt).view(np.uint64)), i
        r = cafs.parse_report(c["report"])
        ro = oracle.report(x, dt)
        for f in oracle.REPORT_FIELDS:
            assert r[f] == ro[f], (i, f, r[f], ro[f])
        uo, co = oracle.counts(x, dt)
        k = r["k_exact"]
        assert np.array_equal(c["uniq"][:k].cpu().numpy().view(np.uint64), uo.view(np.uint64)), i
        assert np.array_equal(c["counts"][:k].cpu().numpy().view(np.uint64), co), i


def test_batch_graph_capture_replays(ctx):
    """A captured batched call replays correctly with new column contents (same
    sizes) copied in between replays, eager batched calls in between too."""
    import paper_2605_25040_amd as cafs
    spec = gen.batch_spec(48, seed=31, n_lo=1e3, n_hi=4e5, k_cap=5e4)
    rounds = []
    for r in range(3):
        rounds.append([gen.column(c["n"], c["k"], dist=c["dist"], s=c["s"], seed=c["seed"] + 977 * r,
                                  dtype=np.uint64) for c in spec])
    m = len(spec)
    cols = make_cols(rounds[0], [True] * m, [True] * m, [True] * m)
    ws = ctx.workspace(ctx.batched_workspace_bytes([c["in"].numel() for c in cols]))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.sort_batched(cols, ws=ws)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            ctx.sort_batched(cols, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for r, arrays in enumerate(rounds + rounds[:1]):
        for c, x in zip(cols, arrays):
            c["in"].copy_(torch.from_numpy(x.view(np.int64).copy()))
            c["src"] = x
        torch.cuda.synchronize()
        g.replay()
        check_cols(cols, "replay %d" % r)
        ctx.sort_batched(cols, ws=ws)
        check_cols(cols, "eager %d" % r)


def test_autotune_and_geometry_extremes(ctx):
    """The autotuner leaves a tuning drawn from its candidates, and outputs, counts
    and reports stay equal to the oracle's under it and under extreme count
    geometries: partitions from an estimate of 512 up, 4-key LDS buckets for every
    estimate, the smallest global tables (so that many keys spill)."""
    spec = gen.batch_spec(96, seed=41, n_lo=1e3, n_hi=2e6, k_cap=6e4)
    arrays = [gen.column(c["n"], c["k"], dist=c["dist"], s=c["s"], seed=c["seed"], dtype=np.uint64) for c in spec]
    m = len(arrays)
    cols = make_cols(arrays, [False] * m, [True] * m, [True] * m)
    try:
        best = ctx.autotune_batched(cols)
        t = ctx.tuning()
        assert best > 0
        assert t["part_keys"] in (4500, 6000, 9000) and t["wide_min"] in (1200, 1800, 2600), t
        assert t["table_slots"] in (16, 32, 64), t
        ctx.sort_batched(cols)
        check_cols(cols, "tuned")
        for geo in (dict(part_keys=256, wide_min=0, table_slots=2), dict(part_keys=100_000, wide_min=1 << 40,
                                                                           table_slots=256)):
            ctx.set_count_geometry(**geo)
            ctx.sort_batched(cols)
            check_cols(cols, "geometry %r" % geo)
            for x in arrays[:12]:
                check_single(ctx, x, False, label="single, geometry %r" % geo)
    finally:
        ctx.set_count_geometry()
        ctx.set_batch_tuning(1 << 16, 1 << 18)
