"""GPU parity at the sizes the workloads are stated at.

Every element of the sorted output, every distinct key and count and every report
field is compared with the oracle (Sec. 6 checks each sort element-wise against a
sorted copy):
  * the HBM-scale column, N = 2^28 int64, K = 1000 Zipf(1.0) over random 64-bit
    values, and its uint64 dictionary-code variant (values 0..999, the same ranks);
  * the dispatcher sweep, N = 3*10^7 int64, K in {4, 8, 200, 10^4, 1.3*10^5,
    6.7*10^5, 3*10^6, N}, uniform and Zipf(1.1) frequencies, one seed;
  * the batched workload, 4096 columns with N log-uniform in [10^3, 10^7] scaled to
    a total of about 2^28 keys, K log-uniform in [2, min(N/2, 10^5)], uniform or
    Zipf(1.1) by a coin, every column checked;
  * the plain column, N = 10^6, K = 200.
The oracle's three passes (sort, counts, report) run in host threads (the oracle
library releases the interpreter lock), beside the GPU work.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_POOL = cf.ThreadPoolExecutor(max_workers=14)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_25040_amd as cafs
    return cafs.Context(0)


def oracle_async(x, dt):
    """Futures of the oracle's sorted copy, (uniq, counts) and report of x."""
    return (_POOL.submit(oracle.sort, x, dt), _POOL.submit(oracle.counts, x, dt),
            _POOL.submit(oracle.report, x, dt))


def sort_on_gpu(ctx, x_np, unsigned):
    """Sorts x on the GPU with counts and report; returns host copies."""
    import paper_2605_25040_amd as cafs
    xi = torch.from_numpy(x_np.view(np.int64)).to("cuda:0")
    out, rep, uq, ct = ctx.sort(xi, unsigned=unsigned, counts=True)
    torch.cuda.synchronize()
    r = cafs.parse_report(rep)
    k = r["k_exact"]
    dt = np.uint64 if unsigned else np.int64
    y = out.cpu().numpy().view(dt)
    u = uq[:k].cpu().numpy().view(dt)
    c = ct[:k].cpu().numpy().view(np.uint64)
    del xi, out, uq, ct
    return y, r, u, c


def compare(label, y, r, u, c, futs):
    f_sort, f_counts, f_rep = futs
    want = f_sort.result()
    assert y.size == want.size, label
    bad = np.flatnonzero(y != want)
    assert bad.size == 0, "%s: %d output elements differ, first at %d" % (label, bad.size, bad[0])
    uo, co = f_counts.result()
    assert np.array_equal(u, uo), "%s: distinct keys differ" % label
    assert np.array_equal(c, co), "%s: counts differ" % label
    ro = f_rep.result()
    for f in oracle.REPORT_FIELDS:
        assert r[f] == ro[f], "%s: report field %s gpu=%r oracle=%r" % (label, f, r[f], ro[f])
    return ro


@pytest.mark.parametrize("variant", ["i64_zipf1.0_random", "u64_codes"])
def test_hbm_scale_column(ctx, variant):
    n, k = 1 << 28, 1000
    if variant == "u64_codes":
        x = gen.column(n, k, dist="zipf", s=1.0, palette="codes", dtype=np.uint64)
        unsigned = True
    else:
        x = gen.column(n, k, dist="zipf", s=1.0, palette="random", dtype=np.int64)
        unsigned = False
    dt = np.uint64 if unsigned else np.int64
    futs = oracle_async(x.view(dt), dt)
    y, r, u, c = sort_on_gpu(ctx, x, unsigned)
    ro = compare("hbm-scale %s" % variant, y, r, u, c, futs)
    assert ro["path"] == "MAIN"
    torch.cuda.empty_cache()


SWEEP_N = 30_000_000
SWEEP_K = [4, 8, 200, 10_000, 130_000, 670_000, 3_000_000, 30_000_000]
SWEEP_DISTS = ["uniform", "zipf"]


@pytest.fixture(scope="module")
def sweep_oracle():
    """Every sweep column and its oracle futures, submitted at once (the largest
    configs take the oracle about a minute), so that the oracle runs ahead of the
    GPU tests."""
    cols = {}
    for k in sorted(SWEEP_K, reverse=True):
        for dist in SWEEP_DISTS:
            x = gen.column(SWEEP_N, k, dist=dist, s=1.1, palette="random", dtype=np.int64)
            cols[(k, dist)] = (x, oracle_async(x, np.int64))
    yield cols
    cols.clear()


@pytest.mark.parametrize("dist", SWEEP_DISTS)
@pytest.mark.parametrize("k", SWEEP_K)
def test_dispatcher_sweep(ctx, sweep_oracle, k, dist):
    x, futs = sweep_oracle[(k, dist)]
    y, r, u, c = sort_on_gpu(ctx, x, False)
    compare("sweep K=%d %s" % (k, dist), y, r, u, c, futs)


def test_plain_column(ctx):
    n, k = 1_000_000, 200
    x = gen.column(n, k, dtype=np.int64)
    futs = oracle_async(x, np.int64)
    y, r, u, c = sort_on_gpu(ctx, x, False)
    ro = compare("plain", y, r, u, c, futs)
    assert ro["path"] == "MAIN"


def test_batched_4096_columns(ctx):
    """The batched workload at its stated size, every column against the oracle."""
    import paper_2605_25040_amd as cafs
    spec = gen.batch_spec(4096, seed=2026, total=1 << 28)
    ns = [c["n"] for c in spec]
    offs = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    flat = np.empty(int(offs[-1]), dtype=np.int64)
    for i, c in enumerate(spec):
        gen.column(c["n"], c["k"], dist=c["dist"], s=c["s"], seed=c["seed"], dtype=np.int64,
                   out=flat[offs[i]:offs[i + 1]].view(np.uint64))
    futs = [oracle_async(flat[offs[i]:offs[i + 1]], np.int64) for i in range(len(spec))]
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(flat).to(dev)
    y = torch.empty_like(x)
    uq = torch.empty_like(x)
    ct = torch.empty_like(x)
    reps = torch.zeros(len(spec), cafs.report_size(), dtype=torch.uint8, device=dev)
    cols = [{"in": x[offs[i]:offs[i + 1]], "out": y[offs[i]:offs[i + 1]], "uniq": uq[offs[i]:offs[i + 1]],
             "counts": ct[offs[i]:offs[i + 1]], "report": reps[i]} for i in range(len(spec))]
    ctx.sort_batched(cols)
    torch.cuda.synchronize()
    y_h = y.cpu().numpy()
    uq_h = uq.cpu().numpy()
    ct_h = ct.cpu().numpy().view(np.uint64)
    reps_h = reps.cpu().numpy()
    del x, y, uq, ct, reps, cols
    torch.cuda.empty_cache()
    paths = {}
    for i in range(len(spec)):
        a, b = offs[i], offs[i + 1]
        r = cafs.parse_report_bytes(reps_h[i].tobytes())
        k = r["k_exact"]
        ro = compare("batch col %d (n=%d k=%d %s)" % (i, ns[i], spec[i]["k"], spec[i]["dist"]),
                     y_h[a:b], r, uq_h[a:a + k], ct_h[a:a + k], futs[i])
        paths[ro["path"]] = paths.get(ro["path"], 0) + 1
    assert sum(paths.values()) == 4096 and paths.get("MAIN", 0) > 1000, paths
