"""Seeded synthetic column generator (host side), shared by tests and bench.

It draws keys only and holds none of the sort's arithmetic.  See
``cafs_gen.c`` for the definition of every distribution and palette.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cafs_gen.c")
_LIB_PATH = os.path.join(_HERE, "libcafs_gen.so")

DISTS = {"uniform": 0, "zipf": 1, "grouped": 2, "runs": 3, "almost_sorted": 4}
PALETTES = {"random": 0, "codes": 1, "ap": 2}


_DEV_SRC = os.path.join(_HERE, "cafs_load.hip")
_DEV_LIB = os.path.join(_HERE, "libcafs_load.so")
_PKG_DIR = os.path.join(os.path.dirname(_HERE), "paper_2605_25040_amd")


def build(force=False):
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_device(force=False):
    """Device generator and serving load driver (needs the built libcafs.so)."""
    if force or not os.path.exists(_DEV_LIB) or \
            os.path.getmtime(_DEV_LIB) < os.path.getmtime(_DEV_SRC):
        tmp = _DEV_LIB + ".tmp"
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
                               "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-o", tmp, _DEV_SRC, "-L" + _PKG_DIR, "-lcafs",
                               "-Wl,-rpath,$ORIGIN/../paper_2605_25040_amd"],
                              stderr=subprocess.DEVNULL)
        os.replace(tmp, _DEV_LIB)
    return _DEV_LIB


_dev = None


def _load_dev():
    global _dev
    if _dev is None:
        if not os.path.exists(_DEV_LIB):
            build_device()
        lib = ctypes.CDLL(_DEV_LIB)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        lib.gen_column_dev.argtypes = [p, u64, u64, ctypes.c_int, ctypes.c_double, ctypes.c_int, u64, p]
        lib.gen_column_dev.restype = ctypes.c_int
        lib.serve_fifo.argtypes = [ctypes.c_int, p, p, p, p, u64, ctypes.c_double, p, p]
        lib.serve_fifo.restype = ctypes.c_int
        lib.copy_dev.argtypes = [p, p, u64, p]
        lib.copy_dev.restype = ctypes.c_int
        lib.serve_replay.argtypes = [ctypes.c_int, p, p, p, p, u64, ctypes.c_double, u64, ctypes.c_uint32,
                                     ctypes.c_uint32, p, p, p, p, p]
        lib.serve_replay.restype = ctypes.c_int
        _dev = lib
    return _dev


def column_device(out, k, dist="uniform", s=1.1, palette="random", seed=None, stream=None):
    """Fill a CUDA int64 tensor on the device (uniform: identical to ``column``;
    zipf: continuous power-law ranks, see cafs_load.hip)."""
    n = out.numel()
    if seed is None:
        seed = default_seed(n, k)
    d = {"uniform": 0, "zipf": 1}[dist]
    rc = _load_dev().gen_column_dev(ctypes.c_void_p(out.data_ptr()), n, int(k), d, float(s), PALETTES[palette],
                                    int(seed) & (2**64 - 1), ctypes.c_void_p(stream) if stream else None)
    if rc != 0:
        raise RuntimeError("gen_column_dev failed: %d" % rc)
    return out


def copy_device(dst, src, stream=None):
    """Plain device copy (16-byte loads, 16-byte nontemporal stores) of src into dst."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    rc = _load_dev().copy_dev(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                              ctypes.c_void_p(stream) if stream else None)
    if rc != 0:
        raise RuntimeError("copy_dev failed: %d" % rc)
    return dst


def serving_trace(rate, seconds, seed=99, n_lo=1e3, n_hi=3e7, k_cap=1e6):
    """Poisson arrivals at ``rate`` per second for ``seconds``; N log-uniform in
    [n_lo, n_hi]; K log-uniform in [2, min(N, k_cap)]; per-request seeds."""
    import math
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * seconds * 1.2) + 16)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    m = t.size
    n = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=m)).astype(np.uint64)
    khi = np.maximum(2.0, np.minimum(n.astype(np.float64), k_cap))
    k = np.exp(rng.uniform(0.0, 1.0, size=m) * np.log(khi / 2.0) + math.log(2.0)).astype(np.uint64)
    k = np.maximum(k, 2)
    seeds = np.array([default_seed(int(a), int(b), column=i) for i, (a, b) in enumerate(zip(n, k))],
                     dtype=np.uint64)
    return t.astype(np.float64), n, k, seeds


def serve_replay(arrival, n, k, seeds, zipf_s=1.1, budget=64 << 30, n_streams=4, max_batch=1024, device=0):
    """Replay a trace through a CAFS server in real time (C++ driver)."""
    m = arrival.size
    arrival = np.ascontiguousarray(arrival, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.uint64)
    k = np.ascontiguousarray(k, dtype=np.uint64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    t_admit = np.zeros(m)
    t_done = np.zeros(m)
    path = np.zeros(m, dtype=np.int32)
    kex = np.zeros(m, dtype=np.uint64)
    stats = np.zeros(10)
    rc = _load_dev().serve_replay(device, arrival.ctypes.data, n.ctypes.data, k.ctypes.data, seeds.ctypes.data, m,
                                  float(zipf_s), int(budget), int(n_streams), int(max_batch), t_admit.ctypes.data,
                                  t_done.ctypes.data, path.ctypes.data, kex.ctypes.data, stats.ctypes.data)
    if rc != 0:
        raise RuntimeError("serve_replay failed: %d" % rc)
    keys = ["wall_s", "keys", "batches", "launched", "refused", "max_busy_streams", "arena_high_water",
            "arena_used", "queued", "max_waiting"]
    return dict(t_admit=t_admit, t_done=t_done, path=path, k_exact=kex, stats=dict(zip(keys, stats.tolist())))


def serve_fifo(arrival, n, k, seeds, zipf_s=1.1, device=0):
    """The trace served one request at a time with plain single-column calls."""
    m = arrival.size
    arrival = np.ascontiguousarray(arrival, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.uint64)
    k = np.ascontiguousarray(k, dtype=np.uint64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    t_done = np.zeros(m)
    stats = np.zeros(2)
    rc = _load_dev().serve_fifo(device, arrival.ctypes.data, n.ctypes.data, k.ctypes.data, seeds.ctypes.data, m,
                                float(zipf_s), t_done.ctypes.data, stats.ctypes.data)
    if rc != 0:
        raise RuntimeError("serve_fifo failed: %d" % rc)
    return dict(t_done=t_done, stats=dict(wall_s=float(stats[0]), keys=float(stats[1])))


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        u64 = ctypes.c_uint64
        lib.gen_mix64.argtypes = [u64]
        lib.gen_mix64.restype = u64
        lib.gen_splitmix.argtypes = [u64, u64]
        lib.gen_splitmix.restype = u64
        lib.gen_palette_value.argtypes = [ctypes.c_int, u64, u64]
        lib.gen_palette_value.restype = u64
        lib.gen_zipf_cdf.argtypes = [ctypes.c_void_p, u64, ctypes.c_double]
        lib.gen_zipf_cdf.restype = ctypes.c_int
        lib.gen_column.argtypes = [ctypes.c_void_p, u64, u64, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int, u64]
        lib.gen_column.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_seed(n, k, rep=0, column=0):
    """The paper's seed convention 42 + N + K, plus 2^32*rep + 2^40*column."""
    return (42 + int(n) + int(k) + (int(rep) << 32) + (int(column) << 40)) & (2**64 - 1)


def column(n, k, dist="uniform", s=1.1, palette="random", seed=None, dtype=np.int64, out=None):
    """Generate one column of ``n`` keys with ``k`` palette values.

    Returns a numpy array of ``dtype`` (int64 or uint64; the bits are the same).
    """
    n, k = int(n), int(k)
    if seed is None:
        seed = default_seed(n, k)
    a = out if out is not None else np.empty(n, dtype=np.uint64)
    if a.size != n or a.dtype.itemsize != 8:
        raise ValueError("out must hold n 64-bit values")
    rc = _load().gen_column(a.ctypes.data if n else None, n, k, DISTS[dist], float(s),
                            PALETTES[palette], int(seed) & (2**64 - 1))
    if rc != 0:
        raise ValueError("bad generator arguments")
    return a.view(dtype)


def mix64(z):
    return int(_load().gen_mix64(int(z) & (2**64 - 1)))


def splitmix(seed, i):
    return int(_load().gen_splitmix(int(seed) & (2**64 - 1), int(i)))


def palette_value(palette, seed, r):
    return int(_load().gen_palette_value(PALETTES[palette], int(seed) & (2**64 - 1), int(r)))


def zipf_cdf(k, s):
    cdf = np.empty(int(k), dtype=np.float64)
    _load().gen_zipf_cdf(cdf.ctypes.data, int(k), float(s))
    return cdf


def batch_spec(n_cols, seed=7, n_lo=1e3, n_hi=1e7, k_cap=1e5, total=None):
    """Column shapes of the batched workload.

    N log-uniform in [n_lo, n_hi]; K log-uniform in [2, min(N/2, k_cap)]; each
    column uniform or Zipf(1.1) frequencies by a fair coin; one seed per column
    (42 + N + K + 2^40 * column).  With ``total`` every N is scaled so that the
    sum is about ``total`` (floor n_lo) and K is re-clipped to N/2.
    Returns a list of dicts (n, k, dist, s, seed).
    """
    import math
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_cols))
    if total is not None:
        ns = np.maximum(n_lo, ns * (float(total) / ns.sum()))
    ns = ns.astype(np.int64)
    out = []
    for i, n in enumerate(ns):
        khi = max(2.0, min(n / 2.0, k_cap))
        k = int(math.exp(rng.uniform(math.log(2.0), math.log(khi)))) if khi > 2 else 2
        dist = "zipf" if rng.random() < 0.5 else "uniform"
        out.append(dict(n=int(n), k=max(2, k), dist=dist, s=1.1, seed=default_seed(n, k, column=i)))
    return out
