"""The allocation-free entry point (cafs_sort_noalloc) against cafs_sort_i64/u64/f64
through the C ABI: bit-identical sorted output, distinct keys, counts and report,
on consecutive calls (the second on a smaller column), plus its size limit."""
import ctypes

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

I64, U64, F64 = 0, 1, 2


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_25040_amd as cafs
    c = cafs.Context(0)
    lib = c._lib
    p, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32
    lib.cafs_sort_noalloc.argtypes = [p, p, p, u64, i32, p, p, p, p]
    lib.cafs_sort_noalloc.restype = i32
    return c


def _stream():
    return torch.cuda.current_stream().cuda_stream


def run_both(ctx, x_np, dtype):
    """Sorts x with the workspace entry point and with the allocation-free one;
    returns both (out, uniq, counts, report bytes) as host copies."""
    import paper_2605_25040_amd as cafs
    lib = ctx._lib
    n = x_np.size
    tdt = torch.float64 if dtype == F64 else torch.int64
    x = torch.from_numpy(x_np.view(np.float64 if dtype == F64 else np.int64).copy()).to("cuda:0")
    res = []
    for which in ("ws", "noalloc"):
        out = torch.full((max(n, 1),), -3, dtype=tdt, device="cuda:0")
        uq = torch.full((max(n, 1),), -5, dtype=tdt, device="cuda:0")
        ct = torch.full((max(n, 1),), -7, dtype=torch.int64, device="cuda:0")
        rep = torch.zeros(cafs.report_size(), dtype=torch.uint8, device="cuda:0")
        if which == "ws":
            fn = {I64: lib.cafs_sort_i64, U64: lib.cafs_sort_u64, F64: lib.cafs_sort_f64}[dtype]
            ws = ctx.workspace(ctx.workspace_bytes(n))
            rc = fn(ctx._h, x.data_ptr(), out.data_ptr(), n, uq.data_ptr(), ct.data_ptr(), rep.data_ptr(),
                    ws.data_ptr(), ws.numel(), _stream())
        else:
            rc = lib.cafs_sort_noalloc(ctx._h, x.data_ptr(), out.data_ptr(), n, dtype, uq.data_ptr(), ct.data_ptr(),
                                       rep.data_ptr(), _stream())
        assert rc == 0, (which, rc)
        torch.cuda.synchronize()
        r = cafs.parse_report(rep)
        k = r["k_exact"]
        res.append((out[:n].cpu().numpy().view(np.uint64), uq[:k].cpu().numpy().view(np.uint64),
                    ct[:k].cpu().numpy().view(np.uint64), r))
    return res


CASES = [
    # (n, k, dist, dtype): two calls in a row, the second smaller
    ((1 << 20, 1000, "zipf", I64), (300_001, 200, "uniform", I64)),
    ((1_000_000, 200, "uniform", U64), (5000, 5, "uniform", U64)),
    ((900_000, 300_000, "uniform", I64), (70_000, 20_000, "uniform", I64)),
    ((600_000, 40_000, "zipf", I64), (2047, 100, "uniform", I64)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_equals_workspace_call(ctx, first, second):
    for n, k, dist, dtype in (first, second):
        x = gen.column(n, k, dist=dist, s=1.1, dtype=np.uint64)
        (y0, u0, c0, r0), (y1, u1, c1, r1) = run_both(ctx, x, dtype)
        assert np.array_equal(y1, y0), (n, k)
        assert np.array_equal(u1, u0) and np.array_equal(c1, c0), (n, k)
        # (engine and flags tell what ran; a spill of a few keys can depend on timing)
        assert all(r1[f] == r0[f] for f in oracle.REPORT_FIELDS), (n, k, r0, r1)
        dt = np.uint64 if dtype == U64 else np.int64
        assert np.array_equal(y1.view(dt), oracle.sort(x.view(dt), dt)), (n, k)


def test_noalloc_float64_and_ragged(ctx):
    rng = np.random.default_rng(4)
    pal = rng.normal(size=300) * 10.0 ** rng.uniform(-20, 20, size=300)
    for n in (400_000, 3):
        x = pal[rng.integers(0, pal.size, size=n)].view(np.uint64)
        (y0, u0, c0, r0), (y1, u1, c1, r1) = run_both(ctx, x, F64)
        assert np.array_equal(y1, y0) and np.array_equal(u1, u0) and np.array_equal(c1, c0)
        assert all(r1[f] == r0[f] for f in oracle.REPORT_FIELDS), (n, r0, r1)


def test_noalloc_limit(ctx):
    lib = ctx._lib
    n = (1 << 20) + 1
    x = torch.zeros(n, dtype=torch.int64, device="cuda:0")
    y = torch.full((n,), 9, dtype=torch.int64, device="cuda:0")
    assert lib.cafs_sort_noalloc(ctx._h, x.data_ptr(), y.data_ptr(), n, I64, None, None, None, _stream()) == -1
    assert lib.cafs_sort_noalloc(None, x.data_ptr(), y.data_ptr(), 10, I64, None, None, None, _stream()) == -1
    assert lib.cafs_sort_noalloc(ctx._h, x.data_ptr(), y.data_ptr(), 10, 5, None, None, None, _stream()) == -1
    torch.cuda.synchronize()
    assert bool((y == 9).all())
    # exactly at the limit works
    n = 1 << 20
    xs = torch.arange(n, 0, -1, dtype=torch.int64, device="cuda:0")
    assert lib.cafs_sort_noalloc(ctx._h, xs.data_ptr(), y.data_ptr(), n, I64, None, None, None, _stream()) == 0
    torch.cuda.synchronize()
    assert torch.equal(y[:n], torch.arange(1, n + 1, dtype=torch.int64, device="cuda:0"))
