"""The C-ABI library loads and exports every entry point include/cafs.h declares.

No compute calls: these run without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cafs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cafs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2605_25040_amd as cafs
    if not os.path.exists(cafs.LIB_PATH):
        from paper_2605_25040_amd import build
        build.build()
    return cafs.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    import paper_2605_25040_amd as cafs
    assert sorted(cafs.EXPORTS) == names


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.cafs_status_str(code)
    assert lib.cafs_status_str(0) == b"ok"


def test_workspace_bytes_grows_with_n(lib):
    prev = 0
    for n in (0, 1, 2047, 2048, 10**5, 10**6, 3 * 10**7, 1 << 28):
        b = lib.cafs_workspace_bytes(n, 0)
        assert b >= prev and b % 256 == 0
        prev = b
    # the radix scratch and the dense arrays scale with n
    assert lib.cafs_workspace_bytes(1 << 28, 0) >= 24 * (1 << 28)


def test_argument_errors_without_gpu(lib):
    p = ctypes.c_void_p
    # NULL context
    assert lib.cafs_sort_i64(None, p(16), p(16), 10, None, None, None, p(256), 1 << 20, None) == -1
    assert lib.cafs_radix_sort(None, p(16), p(16), 10, 0, p(256), 1 << 20, None) == -1
    assert lib.cafs_estimate(None, p(16), 10, 0, p(16), None) == -1
    assert lib.cafs_sort_f64(None, p(16), p(16), 10, None, None, None, p(256), 1 << 20, None) == -1
    assert lib.cafs_ctx_set_hash_seed(None, 5) == -1
    h = ctypes.c_void_p()
    assert lib.cafs_ctx_create(None, 0) == -1


def test_report_layout_matches_header():
    import paper_2605_25040_amd as cafs
    # cafs_estimate_t: 6 u64 + 2 u32 = 56 bytes; cafs_report_t: 56 + 2*i32 + 3*u64 + 2*u32 = 96
    assert ctypes.sizeof(cafs.Estimate) == 56
    assert cafs.report_size() == 96


def test_batched_workspace_is_sum_of_columns(lib):
    import ctypes as ct
    ns = [0, 1, 5000, 10**6, 3 * 10**6]
    arr = (ct.c_uint64 * len(ns))(*ns)
    lib.cafs_batched_workspace_bytes.argtypes = [ct.c_void_p, ct.c_uint32]
    lib.cafs_batched_workspace_bytes.restype = ct.c_size_t
    total = lib.cafs_batched_workspace_bytes(arr, len(ns))
    per = sum(lib.cafs_workspace_bytes(n, 0) for n in ns)
    assert total >= per and total % 256 == 0
    assert total - per < 1 << 20  # the header (arguments and block tables) is small
