"""Error paths of the C ABI with a live context: every rejected call returns its
status before enqueuing anything, so the output buffer keeps its contents."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EINVAL, EWORKSPACE, EUNSUPPORTED = -1, -2, -4


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_25040_amd as cafs
    return cafs.Context(0)


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _sort(ctx, x_ptr, y_ptr, n, ws_ptr, ws_bytes, uniq=None, counts=None, report=None, fn="cafs_sort_i64"):
    return getattr(ctx._lib, fn)(ctx._h, x_ptr, y_ptr, n, uniq, counts, report, ws_ptr, ws_bytes, _stream())


def test_workspace_errors(ctx):
    n = 100_000
    x = torch.arange(n, 0, -1, dtype=torch.int64, device="cuda:0")
    y = torch.full((n,), 7, dtype=torch.int64, device="cuda:0")
    need = ctx.workspace_bytes(n)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda:0")
    base = ws.data_ptr()
    assert base % 256 == 0
    # too small by one byte
    assert _sort(ctx, x.data_ptr(), y.data_ptr(), n, base, need - 1) == EWORKSPACE
    # no workspace
    assert _sort(ctx, x.data_ptr(), y.data_ptr(), n, None, need) == EWORKSPACE
    # large enough but not 256-byte aligned (8, 64 and 128 bytes off)
    for off in (8, 64, 128):
        assert _sort(ctx, x.data_ptr(), y.data_ptr(), n, base + off, need) == EWORKSPACE
    assert ctx._lib.cafs_radix_sort(ctx._h, x.data_ptr(), y.data_ptr(), n, 0, base + 64, need, _stream()) \
        == EWORKSPACE
    torch.cuda.synchronize()
    assert bool((y == 7).all()), "a rejected call wrote the output"
    # the exact size works
    assert _sort(ctx, x.data_ptr(), y.data_ptr(), n, base, need) == 0
    torch.cuda.synchronize()
    assert torch.equal(y, torch.arange(1, n + 1, dtype=torch.int64, device="cuda:0"))


def test_overlap_and_alignment_errors(ctx):
    n = 50_000
    buf = torch.zeros(3 * n, dtype=torch.int64, device="cuda:0")
    buf[:n] = torch.arange(n, 0, -1, device="cuda:0")
    need = ctx.workspace_bytes(2 * n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    p = buf.data_ptr()
    # output overlapping the input in part, in both directions
    for shift in (1, n - 1, -1, -(n - 1)):
        xin = p + (n if shift < 0 else 0) * 8
        yout = xin + shift * 8
        assert _sort(ctx, xin, yout, n, ws.data_ptr(), need) == EINVAL, shift
    # keys not 8-byte aligned
    assert _sort(ctx, p + 4, p + 2 * n * 8, n, ws.data_ptr(), need) == EINVAL
    assert _sort(ctx, p, p + 2 * n * 8 + 4, n, ws.data_ptr(), need) == EINVAL
    # n > 0 with a null pointer
    assert _sort(ctx, None, p + 2 * n * 8, n, ws.data_ptr(), need) == EINVAL
    assert _sort(ctx, p, None, n, ws.data_ptr(), need) == EINVAL
    # n >= 2^32
    assert _sort(ctx, p, p + 2 * n * 8, 1 << 32, ws.data_ptr(), need) == EINVAL
    # counts requested without a report
    assert _sort(ctx, p, p + 2 * n * 8, n, ws.data_ptr(), need, counts=p + n * 8) == EINVAL
    # unknown dtype (radix API and estimate)
    assert ctx._lib.cafs_radix_sort(ctx._h, p, p + 2 * n * 8, n, 7, ws.data_ptr(), need, _stream()) == EINVAL
    est = torch.zeros(64, dtype=torch.uint8, device="cuda:0")
    assert ctx._lib.cafs_estimate(ctx._h, p, n, 7, est.data_ptr(), _stream()) == EINVAL
    assert ctx._lib.cafs_estimate(ctx._h, p + 4, n, 0, est.data_ptr(), _stream()) == EINVAL
    # 32-bit keys need 4-byte alignment only, but not 2
    assert _sort(ctx, p + 2, p + 2 * n * 8, n, ws.data_ptr(), need, fn="cafs_sort_i32") == EINVAL
    assert _sort(ctx, p, p + 2 * n * 8 + 2, n, ws.data_ptr(), need, fn="cafs_sort_u32") == EINVAL
    assert ctx._lib.cafs_estimate(ctx._h, p + 2, n, 3, est.data_ptr(), _stream()) == EINVAL
    # a 32-bit output overlapping the input by one key
    assert _sort(ctx, p, p + 4, n, ws.data_ptr(), need, fn="cafs_sort_i32") == EINVAL
    torch.cuda.synchronize()
    assert bool((buf[n:] == 0).all()), "a rejected call wrote memory"
    # in place is allowed
    assert _sort(ctx, p, p, n, ws.data_ptr(), need) == 0
    torch.cuda.synchronize()
    assert torch.equal(buf[:n], torch.arange(1, n + 1, dtype=torch.int64, device="cuda:0"))


def test_batched_errors(ctx):
    import paper_2605_25040_amd as cafs
    n = 10_000
    x = torch.arange(n, 0, -1, dtype=torch.int64, device="cuda:0")
    y = torch.zeros(n, dtype=torch.int64, device="cuda:0")
    cols = [{"in": x, "out": y}]
    arr = ctx._columns(cols)
    need = ctx.batched_workspace_bytes([n])
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda:0")
    lib = ctx._lib
    assert lib.cafs_sort_batched(ctx._h, arr, 1, ws.data_ptr(), need - 1, _stream()) == EWORKSPACE
    assert lib.cafs_sort_batched(ctx._h, arr, 1, ws.data_ptr() + 128, need, _stream()) == EWORKSPACE
    arr[0].flags = 1
    assert lib.cafs_sort_batched(ctx._h, arr, 1, ws.data_ptr(), need, _stream()) == EINVAL
    arr[0].flags = 0
    arr[0].dtype = 9
    assert lib.cafs_sort_batched(ctx._h, arr, 1, ws.data_ptr(), need, _stream()) == EINVAL
    arr[0].dtype = 0
    arr[0].d_out = x.data_ptr() + 8  # partial overlap
    assert lib.cafs_sort_batched(ctx._h, arr, 1, ws.data_ptr(), need, _stream()) == EINVAL
    arr[0].d_out = y.data_ptr()
    arr[0].d_counts = y.data_ptr()  # counts without a report
    assert lib.cafs_sort_batched(ctx._h, arr, 1, ws.data_ptr(), need, _stream()) == EINVAL
    arr[0].d_counts = None
    torch.cuda.synchronize()
    assert bool((y == 0).all())
    assert lib.cafs_sort_batched(ctx._h, arr, 1, ws.data_ptr(), need, _stream()) == 0
    torch.cuda.synchronize()
    assert torch.equal(y, torch.arange(1, n + 1, dtype=torch.int64, device="cuda:0"))
    assert cafs.report_size() == ctypes.sizeof(cafs.Report)
    # status strings name every code
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.cafs_status_str(code).decode() not in ("", "unknown status")


def test_empty_column_report(ctx):
    import paper_2605_25040_amd as cafs
    rep = torch.full((cafs.report_size(),), 0xAB, dtype=torch.uint8, device="cuda:0")
    assert _sort(ctx, None, None, 0, None, 0, report=rep.data_ptr()) == 0
    torch.cuda.synchronize()
    r = cafs.parse_report(rep)
    assert r["path"] == "MONOTONE" and r["k_exact"] == 0 and r["k_hat"] == 0
