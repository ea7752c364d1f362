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


def build(force=False):
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


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
