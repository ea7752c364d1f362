"""CAFS reference oracle (test infrastructure only).

Thin ctypes wrapper around ``liboracle.so`` built from ``cafs_oracle.cpp``.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the GPU library never does, and shares no code with it.

Report fields follow the dispatcher of Alg. 3 and the reconstruction of Alg. 4
of the CAFS paper: the Chao1 estimate (Alg. 2), the path label, the tiny-count
miss flag, the bucket count M (Eq. Msize), the spill size in elements and the
exact number of distinct keys.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cafs_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

PATHS = ("MONOTONE", "SMALL_N", "TINY", "HIGH_K", "MAIN", "GUARD")
REPORT_FIELDS = ("k_hat", "u", "f1", "f2", "n_samples", "stride", "saturated",
                 "path", "tiny_miss", "table_M", "spill_elems", "k_exact")
ESTIMATE_FIELDS = REPORT_FIELDS[:7]


def build(force=False):
    """Compile the oracle with g++ (plain C++17, no GPU code)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p, u64 = ctypes.c_void_p, ctypes.c_uint64
        for name in ("oracle_sort_i64", "oracle_sort_u64", "oracle_sort_f64", "oracle_std_sort_i64",
                     "oracle_sort_i32", "oracle_sort_u32"):
            getattr(lib, name).argtypes = [p, u64, p]
            getattr(lib, name).restype = None
        for name in ("oracle_counts_i64", "oracle_counts_u64", "oracle_counts_f64", "oracle_counts_i32",
                     "oracle_counts_u32"):
            getattr(lib, name).argtypes = [p, u64, p, p]
            getattr(lib, name).restype = u64
        for name in ("oracle_is_monotone_i64", "oracle_is_monotone_u64", "oracle_is_monotone_f64",
                     "oracle_is_monotone_i32", "oracle_is_monotone_u32"):
            getattr(lib, name).argtypes = [p, u64]
            getattr(lib, name).restype = ctypes.c_int
        for name in ("oracle_estimate", "oracle_report_i64", "oracle_report_u64", "oracle_report_f64",
                     "oracle_report_i32", "oracle_report_u32"):
            getattr(lib, name).argtypes = [p, u64, p]
            getattr(lib, name).restype = None
        for name in ("oracle_table_M", "oracle_table_M32"):
            getattr(lib, name).argtypes = [u64, u64]
            getattr(lib, name).restype = u64
        for name in ("oracle_sort_kv_i64", "oracle_sort_kv_u64", "oracle_sort_kv_f64", "oracle_sort_kv_i32",
                     "oracle_sort_kv_u32"):
            getattr(lib, name).argtypes = [p, p, u64, p, p]
            getattr(lib, name).restype = None
        lib.oracle_hash.argtypes = [u64, u64]
        lib.oracle_hash.restype = u64
        for name in ("oracle_spill", "oracle_spill32"):
            getattr(lib, name).argtypes = [p, u64, u64]
            getattr(lib, name).restype = u64
        _lib = lib
    return _lib


def _arr(x, dtype):
    a = np.ascontiguousarray(x)
    if a.dtype != dtype:
        if a.dtype.itemsize != np.dtype(dtype).itemsize or a.dtype.kind not in "iuf":
            raise TypeError("oracle takes 64-bit or 32-bit integer or float64 arrays of the dtype's width")
        a = a.view(dtype)
    return a


def _kind(dtype):
    """Suffix of the oracle function for ``dtype``: int64, uint64, float64 (IEEE 754
    totalOrder on the bit patterns), int32 or uint32."""
    d = np.dtype(dtype)
    return {("i", 8): "i64", ("u", 8): "u64", ("f", 8): "f64", ("i", 4): "i32", ("u", 4): "u32"}[(d.kind, d.itemsize)]


def _ptr(a):
    return a.ctypes.data if a.size else None


def sort(x, dtype=np.int64):
    """Sorted copy of ``x`` (nondecreasing in ``dtype``'s order)."""
    a = _arr(x, dtype)
    y = np.empty_like(a)
    getattr(_load(), "oracle_sort_" + _kind(dtype))(_ptr(a), a.size, _ptr(y))
    return y


def sort_kv(x, v, dtype=np.int64):
    """Stable key-value sort: (keys in ``dtype``'s order, the 64-bit payloads ``v``
    moved with their keys, equal keys in input order)."""
    a = _arr(x, dtype)
    vals = np.ascontiguousarray(v).view(np.uint64)
    if vals.shape != a.shape:
        raise ValueError("one 64-bit payload per key")
    y = np.empty_like(a)
    w = np.empty_like(vals)
    getattr(_load(), "oracle_sort_kv_" + _kind(dtype))(_ptr(a), _ptr(vals), a.size, _ptr(y), _ptr(w))
    return y, w


def std_sort_i64(x):
    """Sorted copy of an int64 array by a plain single-thread std::sort."""
    a = _arr(x, np.int64)
    y = np.empty_like(a)
    _load().oracle_std_sort_i64(_ptr(a), a.size, _ptr(y))
    return y


def counts(x, dtype=np.int64):
    """(uniq, counts) of ``x`` with ``uniq`` ascending in ``dtype``'s order."""
    a = _arr(x, dtype)
    uniq = np.empty_like(a)
    cnt = np.empty(a.size, dtype=np.uint64)
    k = getattr(_load(), "oracle_counts_" + _kind(dtype))(_ptr(a), a.size, _ptr(uniq), _ptr(cnt))
    return uniq[:k].copy(), cnt[:k].copy()


def is_monotone(x, dtype=np.int64):
    a = _arr(x, dtype)
    return bool(getattr(_load(), "oracle_is_monotone_" + _kind(dtype))(_ptr(a), a.size))


def estimate(x):
    """Chao1 estimate over 1024 strided samples (Alg. 2), as a dict."""
    a = _arr(x, np.uint64)
    out = np.zeros(7, dtype=np.uint64)
    _load().oracle_estimate(_ptr(a), a.size, _ptr(out))
    return {k: int(v) for k, v in zip(ESTIMATE_FIELDS, out)}


def table_M(k_hat, n, cap=4):
    """Bucket count of Eq. Msize (cap 4 for 64-bit keys, 8 for 32-bit keys; clamped
    to [8, bit_ceil(N/cap)])."""
    fn = {4: _load().oracle_table_M, 8: _load().oracle_table_M32}[cap]
    return int(fn(int(k_hat), int(n)))


def hash_bucket(v, M):
    """Eq. hash: top log2(M) bits of v * 0x9E3779B97F4A7C15 mod 2^64."""
    return int(_load().oracle_hash(int(v) & (2**64 - 1), int(M)))


def spill(x, M, cap=4):
    """Literal bucket simulation (Alg. 1 + RLE) with buckets of `cap` keys over the
    64-bit values x: spilled element count."""
    a = _arr(x, np.uint64)
    fn = {4: _load().oracle_spill, 8: _load().oracle_spill32}[cap]
    return int(fn(_ptr(a), a.size, int(M)))


def report(x, dtype=np.int64):
    """Full dispatcher report (Alg. 3 + Alg. 4) as a dict with a path name."""
    a = _arr(x, dtype)
    out = np.zeros(12, dtype=np.uint64)
    getattr(_load(), "oracle_report_" + _kind(dtype))(_ptr(a), a.size, _ptr(out))
    r = {k: int(v) for k, v in zip(REPORT_FIELDS, out)}
    r["path"] = PATHS[r["path"]]
    return r
