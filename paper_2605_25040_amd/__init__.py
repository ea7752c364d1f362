"""Python binding of the MI355X CAFS library (libcafs.so, C ABI in include/cafs.h).

Argument marshalling only: every step of the sort runs in the HIP kernels.
PyTorch provides device memory and streams.  The library must have been built
(``python -m paper_2605_25040_amd.build``); there is no CPU fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcafs.so")

PATHS = ("MONOTONE", "SMALL_N", "TINY", "HIGH_K", "MAIN", "GUARD")
ENGINES = ("NONE", "TINY", "HASH", "RADIX")
I64, U64, F64, I32, U32 = 0, 1, 2, 3, 4
STATUS = {0: "ok", -1: "invalid argument", -2: "workspace", -3: "HIP error", -4: "unsupported", -5: "nomem",
          -6: "busy"}

STAGES = ("pre", "count", "order", "emit", "tail")

EXPORTS = ("cafs_ctx_create", "cafs_ctx_destroy", "cafs_ctx_enable_timing", "cafs_ctx_stage_ms",
           "cafs_workspace_bytes", "cafs_estimate",
           "cafs_sort_i64", "cafs_sort_u64", "cafs_sort_f64", "cafs_sort_i32", "cafs_sort_u32", "cafs_sort_kv", "cafs_sort_noalloc", "cafs_radix_sort", "cafs_batched_workspace_bytes",
           "cafs_sort_batched", "cafs_ctx_set_batch_tuning", "cafs_autotune_batched", "cafs_ctx_set_hash_seed", "cafs_ctx_set_count_geometry", "cafs_ctx_get_tuning",
           "cafs_server_create", "cafs_server_destroy", "cafs_server_reserve", "cafs_server_submit",
           "cafs_server_poll", "cafs_server_release", "cafs_server_stats",
           "cafs_status_str", "cafs_last_error")
EBUSY = -6


class Estimate(ctypes.Structure):
    _fields_ = [("k_hat", ctypes.c_uint64), ("u", ctypes.c_uint64), ("f1", ctypes.c_uint64),
                ("f2", ctypes.c_uint64), ("n_samples", ctypes.c_uint64), ("stride", ctypes.c_uint64),
                ("saturated", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class Report(ctypes.Structure):
    _fields_ = [("est", Estimate), ("path", ctypes.c_int32), ("tiny_miss", ctypes.c_int32),
                ("table_M", ctypes.c_uint64), ("spill_elems", ctypes.c_uint64), ("k_exact", ctypes.c_uint64),
                ("engine", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Column(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("d_out", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("dtype", ctypes.c_int32), ("flags", ctypes.c_int32), ("d_uniq", ctypes.c_void_p),
                ("d_counts", ctypes.c_void_p), ("d_report", ctypes.c_void_p)]


class CafsError(RuntimeError):
    pass


_lib = None


def load():
    """Load libcafs.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CafsError("libcafs.so is not built; run `python -m paper_2605_25040_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    p, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32
    lib.cafs_ctx_create.argtypes = [ctypes.POINTER(p), ctypes.c_int]
    lib.cafs_ctx_create.restype = i32
    lib.cafs_ctx_destroy.argtypes = [p]
    lib.cafs_ctx_destroy.restype = None
    lib.cafs_ctx_enable_timing.argtypes = [p, ctypes.c_int]
    lib.cafs_ctx_enable_timing.restype = i32
    lib.cafs_ctx_stage_ms.argtypes = [p, ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.cafs_ctx_stage_ms.restype = i32
    lib.cafs_workspace_bytes.argtypes = [u64, i32]
    lib.cafs_workspace_bytes.restype = ctypes.c_size_t
    lib.cafs_estimate.argtypes = [p, p, u64, i32, p, p]
    lib.cafs_estimate.restype = i32
    for name in ("cafs_sort_i64", "cafs_sort_u64", "cafs_sort_f64", "cafs_sort_i32", "cafs_sort_u32"):
        getattr(lib, name).argtypes = [p, p, p, u64, p, p, p, p, ctypes.c_size_t, p]
        getattr(lib, name).restype = i32
    lib.cafs_sort_kv.argtypes = [p, p, p, p, p, u64, i32, p, p, p, p, ctypes.c_size_t, p]
    lib.cafs_sort_kv.restype = i32
    lib.cafs_sort_noalloc.argtypes = [p, p, p, u64, i32, p, p, p, p]
    lib.cafs_sort_noalloc.restype = i32
    lib.cafs_radix_sort.argtypes = [p, p, p, u64, i32, p, ctypes.c_size_t, p]
    lib.cafs_radix_sort.restype = i32
    lib.cafs_batched_workspace_bytes.argtypes = [p, u32]
    lib.cafs_batched_workspace_bytes.restype = ctypes.c_size_t
    lib.cafs_sort_batched.argtypes = [p, p, u32, p, ctypes.c_size_t, p]
    lib.cafs_sort_batched.restype = i32
    lib.cafs_ctx_set_batch_tuning.argtypes = [p, u64, u64]
    lib.cafs_ctx_set_batch_tuning.restype = i32
    lib.cafs_ctx_set_count_geometry.argtypes = [p, u64, u64, u64]
    lib.cafs_ctx_set_count_geometry.restype = i32
    lib.cafs_ctx_get_tuning.argtypes = [p, ctypes.POINTER(u64), u32]
    lib.cafs_ctx_get_tuning.restype = i32
    lib.cafs_ctx_set_hash_seed.argtypes = [p, u64]
    lib.cafs_ctx_set_hash_seed.restype = i32
    lib.cafs_autotune_batched.argtypes = [p, p, u32, p, ctypes.c_size_t, p, ctypes.POINTER(ctypes.c_double)]
    lib.cafs_autotune_batched.restype = i32
    lib.cafs_server_create.argtypes = [p, ctypes.c_size_t, u32, u32, ctypes.POINTER(p)]
    lib.cafs_server_create.restype = i32
    lib.cafs_server_destroy.argtypes = [p]
    lib.cafs_server_destroy.restype = None
    lib.cafs_server_reserve.argtypes = [p, u64, i32, ctypes.POINTER(u64), ctypes.POINTER(p), ctypes.POINTER(p),
                                        ctypes.POINTER(p)]
    lib.cafs_server_reserve.restype = i32
    lib.cafs_server_submit.argtypes = [p, u64, p, p]
    lib.cafs_server_submit.restype = i32
    lib.cafs_server_poll.argtypes = [p, ctypes.POINTER(u64), u32, ctypes.POINTER(u32)]
    lib.cafs_server_poll.restype = i32
    lib.cafs_server_release.argtypes = [p, u64]
    lib.cafs_server_release.restype = i32
    lib.cafs_server_stats.argtypes = [p, ctypes.POINTER(u64), u32]
    lib.cafs_server_stats.restype = i32
    lib.cafs_status_str.argtypes = [i32]
    lib.cafs_status_str.restype = ctypes.c_char_p
    lib.cafs_last_error.argtypes = []
    lib.cafs_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        lib = load()
        msg = lib.cafs_status_str(rc).decode()
        detail = lib.cafs_last_error().decode()
        raise CafsError("cafs error %d (%s) %s" % (rc, msg, detail))


def _dtype_code(x, unsigned):
    """The cafs_dtype_t of a tensor: float64, int64 (uint64 keys when `unsigned`),
    int32 (uint32 keys when `unsigned`)."""
    if x.dtype == torch.float64:
        return F64
    if x.dtype == torch.int32:
        return U32 if unsigned else I32
    return U64 if unsigned else I64


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A device context (compute-unit count) plus a cached workspace."""

    def __init__(self, device=0):
        if not torch.cuda.is_available():
            raise CafsError("no GPU visible: the CAFS library runs on the GPU only")
        self.device = torch.device("cuda", device)
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.cafs_ctx_create(ctypes.byref(h), device))
        self._h = h
        self._ws = None

    def close(self):
        if self._h:
            self._lib.cafs_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def enable_timing(self, on=True):
        _check(self._lib.cafs_ctx_enable_timing(self._h, 1 if on else 0))

    def stage_ms(self):
        """Summed per-stage milliseconds of the calls recorded since the last read."""
        arr = (ctypes.c_float * len(STAGES))()
        calls = ctypes.c_int()
        _check(self._lib.cafs_ctx_stage_ms(self._h, arr, len(STAGES), ctypes.byref(calls)))
        return {k: float(v) for k, v in zip(STAGES, arr)}, int(calls.value)

    def workspace_bytes(self, n):
        return int(self._lib.cafs_workspace_bytes(int(n), 0))

    def workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def estimate(self, x, unsigned=False):
        """Chao1 estimate of x (int64, int32 or float64 tensor; ``unsigned`` names an
        integer tensor holding unsigned keys) as a dict."""
        out = torch.zeros(ctypes.sizeof(Estimate), dtype=torch.uint8, device=self.device)
        dt = _dtype_code(x, unsigned)
        _check(self._lib.cafs_estimate(self._h, _ptr(x), x.numel(), dt, _ptr(out), _stream(self.device)))
        e = Estimate.from_buffer_copy(bytes(out.cpu().numpy()))
        return {k: int(getattr(e, k)) for k, _ in Estimate._fields_ if k != "pad"}

    def sort(self, x, unsigned=False, out=None, counts=False, report=True, ws=None):
        """Sort a 1-D int64 or int32 tensor on the GPU (unsigned order if
        ``unsigned``), or a float64 tensor in IEEE 754 totalOrder.

        Returns (out, report_tensor, uniq, counts); uniq/counts are None unless
        ``counts``.  Call ``parse_report`` on the report tensor after a sync.
        """
        n = x.numel()
        if x.dtype not in (torch.int64, torch.float64, torch.int32) or not x.is_cuda:
            raise CafsError("sort takes a CUDA int64, int32 or float64 tensor")
        if out is None:
            out = torch.empty_like(x)
        rep = torch.zeros(ctypes.sizeof(Report), dtype=torch.uint8, device=self.device) if (report or counts) else None
        uq = torch.empty_like(x) if counts else None
        ct = torch.empty(n, dtype=torch.int64, device=x.device) if counts else None
        if ws is None:
            ws = self.workspace(self.workspace_bytes(n))
        fn = {F64: self._lib.cafs_sort_f64, U64: self._lib.cafs_sort_u64, I64: self._lib.cafs_sort_i64,
              U32: self._lib.cafs_sort_u32, I32: self._lib.cafs_sort_i32}[_dtype_code(x, unsigned)]
        _check(fn(self._h, _ptr(x), _ptr(out), n, _ptr(uq), _ptr(ct), _ptr(rep), _ptr(ws), ws.numel(),
                  _stream(self.device)))
        return out, rep, uq, ct

    def sort_kv(self, keys, vals, unsigned=False, out_keys=None, out_vals=None, counts=False, report=True,
                ws=None):
        """Stable key-value sort: ``keys`` (int64, int32 or float64; ``unsigned`` as
        for ``sort``) with one 64-bit payload each in ``vals`` (an int64 tensor).
        Returns (keys_out, vals_out, report_tensor, uniq, counts)."""
        n = keys.numel()
        if keys.dtype not in (torch.int64, torch.float64, torch.int32) or not keys.is_cuda:
            raise CafsError("sort_kv takes a CUDA int64, int32 or float64 key tensor")
        if vals.numel() != n or vals.element_size() != 8 or not vals.is_cuda:
            raise CafsError("sort_kv takes one 64-bit payload per key")
        if out_keys is None:
            out_keys = torch.empty_like(keys)
        if out_vals is None:
            out_vals = torch.empty_like(vals)
        rep = torch.zeros(ctypes.sizeof(Report), dtype=torch.uint8, device=self.device) if (report or counts) else None
        uq = torch.empty_like(keys) if counts else None
        ct = torch.empty(n, dtype=torch.int64, device=keys.device) if counts else None
        if ws is None:
            ws = self.workspace(self.workspace_bytes(n))
        _check(self._lib.cafs_sort_kv(self._h, _ptr(keys), _ptr(out_keys), _ptr(vals), _ptr(out_vals), n,
                                      _dtype_code(keys, unsigned), _ptr(uq), _ptr(ct), _ptr(rep), _ptr(ws),
                                      ws.numel(), _stream(self.device)))
        return out_keys, out_vals, rep, uq, ct

    def radix_sort(self, x, unsigned=False, out=None, ws=None):
        n = x.numel()
        if out is None:
            out = torch.empty_like(x)
        if ws is None:
            ws = self.workspace(self.workspace_bytes(n))
        dt = _dtype_code(x, unsigned)
        _check(self._lib.cafs_radix_sort(self._h, _ptr(x), _ptr(out), n, dt, _ptr(ws),
                                         ws.numel(), _stream(self.device)))
        return out

    def batched_workspace_bytes(self, ns):
        arr = (ctypes.c_uint64 * len(ns))(*[int(v) for v in ns])
        return int(self._lib.cafs_batched_workspace_bytes(arr, len(ns)))

    def _columns(self, cols):
        arr = (Column * len(cols))()
        for i, cdesc in enumerate(cols):
            arr[i].d_in = cdesc["in"].data_ptr()
            arr[i].d_out = cdesc["out"].data_ptr()
            arr[i].n = cdesc["in"].numel()
            arr[i].dtype = _dtype_code(cdesc["in"], cdesc.get("unsigned"))
            arr[i].flags = 0
            arr[i].d_uniq = cdesc["uniq"].data_ptr() if cdesc.get("uniq") is not None else None
            arr[i].d_counts = cdesc["counts"].data_ptr() if cdesc.get("counts") is not None else None
            arr[i].d_report = cdesc["report"].data_ptr() if cdesc.get("report") is not None else None
        return arr

    def sort_batched(self, cols, ws=None):
        """cols: list of dicts with keys in, out, unsigned, uniq, counts, report (tensors or None)."""
        arr = self._columns(cols)
        if ws is None:
            ws = self.workspace(self.batched_workspace_bytes([c["in"].numel() for c in cols]))
        _check(self._lib.cafs_sort_batched(self._h, arr, len(cols), _ptr(ws), ws.numel(), _stream(self.device)))

    def set_batch_tuning(self, elems_per_block, elems_per_hash_block):
        _check(self._lib.cafs_ctx_set_batch_tuning(self._h, int(elems_per_block), int(elems_per_hash_block)))

    def set_count_geometry(self, part_keys=6000, wide_min=1800, table_slots=32):
        """Hash-count geometry (speed only): keys per partition, the 4-key bucket
        threshold per partition and global table slots per estimated key."""
        _check(self._lib.cafs_ctx_set_count_geometry(self._h, int(part_keys), int(wide_min), int(table_slots)))

    TUNING = ("batch_elems_per_block", "batch_elems_per_hash_block", "part_keys", "wide_min", "table_slots")

    def tuning(self):
        """The context's batched block sizing and count geometry (as the autotuner left them)."""
        arr = (ctypes.c_uint64 * len(self.TUNING))()
        _check(self._lib.cafs_ctx_get_tuning(self._h, arr, len(self.TUNING)))
        return {k: int(v) for k, v in zip(self.TUNING, arr)}

    def set_hash_seed(self, seed):
        """Seed of the count tables' hash (0: the paper's multiplier)."""
        _check(self._lib.cafs_ctx_set_hash_seed(self._h, int(seed) & (2**64 - 1)))

    def autotune_batched(self, cols, ws=None):
        arr = self._columns(cols)
        if ws is None:
            ws = self.workspace(self.batched_workspace_bytes([c["in"].numel() for c in cols]))
        best = ctypes.c_double()
        _check(self._lib.cafs_autotune_batched(self._h, arr, len(cols), _ptr(ws), ws.numel(), _stream(self.device),
                                               ctypes.byref(best)))
        return best.value


class Server:
    """Continuous-batching server over one context (see include/cafs.h)."""

    STATS = ("batches", "launched", "refused", "max_busy_streams", "arena_high_water", "arena_used", "queued")

    def __init__(self, ctx, hbm_budget, n_streams=4, max_batch=1024):
        self.ctx = ctx
        self._lib = ctx._lib
        h = ctypes.c_void_p()
        _check(self._lib.cafs_server_create(ctx._h, int(hbm_budget), int(n_streams), int(max_batch), ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            self._lib.cafs_server_destroy(self._h)
            self._h = None

    def reserve(self, n, unsigned=False, buffers=False):
        """Returns (ticket, d_in, d_out, d_report) or None when the budget is full."""
        t = ctypes.c_uint64()
        pi, po, pr = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        args = (ctypes.byref(pi), ctypes.byref(po), ctypes.byref(pr)) if buffers else (None, None, None)
        rc = self._lib.cafs_server_reserve(self._h, int(n), U64 if unsigned else I64, ctypes.byref(t), *args)
        if rc == EBUSY:
            return None
        _check(rc)
        return int(t.value), pi.value, po.value, pr.value

    def submit(self, ticket, col=None):
        arr = self.ctx._columns([col]) if col is not None else None
        _check(self._lib.cafs_server_submit(self._h, int(ticket), arr, _stream(self.ctx.device)))

    def poll(self, cap=4096):
        buf = (ctypes.c_uint64 * cap)()
        k = ctypes.c_uint32()
        _check(self._lib.cafs_server_poll(self._h, buf, cap, ctypes.byref(k)))
        return [int(buf[i]) for i in range(k.value)]

    def release(self, ticket):
        _check(self._lib.cafs_server_release(self._h, int(ticket)))

    def stats(self):
        arr = (ctypes.c_uint64 * len(self.STATS))()
        _check(self._lib.cafs_server_stats(self._h, arr, len(self.STATS)))
        return {k: int(v) for k, v in zip(self.STATS, arr)}


def parse_report(rep):
    """Report tensor (device, after a sync) -> dict with the oracle's field names."""
    return parse_report_bytes(bytes(rep.cpu().numpy()))


def parse_report_bytes(raw):
    """A report's bytes (host copy) -> dict with the oracle's field names."""
    r = Report.from_buffer_copy(raw)
    d = {k: int(getattr(r.est, k)) for k, _ in Estimate._fields_ if k != "pad"}
    d.update(path=PATHS[r.path], tiny_miss=int(r.tiny_miss), table_M=int(r.table_M),
             spill_elems=int(r.spill_elems), k_exact=int(r.k_exact), engine=ENGINES[r.engine],
             flags=int(r.flags))
    return d


def report_size():
    return ctypes.sizeof(Report)


def report_fixed_bytes():
    """Bytes of a report that are a function of the column alone (the estimate, path,
    tiny miss, table M, spill and K); the engine and flags words after them record
    what ran."""
    return Report.engine.offset
