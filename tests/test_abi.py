"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every function
that include/cskv.h declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2603_17168_amd import cskv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = ""
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            with open(os.path.join(ROOT, "include", name)) as f:
                text += f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cskv_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = cskv.lib()
    names = declared_functions()
    assert len(names) >= 15
    assert "cskv_mt_run" in names and "cskv_create_tiered" in names
    for n in names:
        assert hasattr(lib, n), n


def test_table_bytes():
    lib = cskv.lib()
    nb, dim = 2048, 8
    got = lib.cskv_table_bytes(nb * 128, 128, dim)
    # digests + keys + scores + rows per slot, plus 24 bytes per bucket (operation counts and the
    # cached minimum; each array 256-aligned)
    expect = nb * 128 * (1 + 8 + 8 + 4 * dim) + nb * 24
    assert expect <= got <= expect + 6 * 256
    assert lib.cskv_table_bytes(0, 128, 8) == 0
    assert lib.cskv_table_bytes(128 * 6, 128, 8) == 0  # 6 buckets
    assert lib.cskv_table_bytes(128 * 4, 128, 0) == 0
    assert lib.cskv_table_bytes(128 * 4, 128, 1028) == 0
    assert lib.cskv_table_bytes(128 * (1 << 25), 128, 4) == 0  # more than 2^24 buckets
    assert lib.cskv_table_bytes(128 * (1 << 24), 128, 4) > 0


def test_create_rejects_bad_arguments_without_device_work():
    lib = cskv.lib()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails validation first
    big = 1 << 40
    assert lib.cskv_create(None, 128 * 4, 128, 8, 2, 0, fake, big, None) == -1
    assert lib.cskv_create(ctypes.byref(h), 128 * 4, 128, 8, 3, 0, fake, big, None) == -1  # mode
    assert lib.cskv_create(ctypes.byref(h), 128 * 4, 128, 8, 2, 9, fake, big, None) == -1  # policy
    assert lib.cskv_create(ctypes.byref(h), 128 * 4, 64, 8, 2, 0, fake, big, None) == -4  # bucket size
    assert lib.cskv_create(ctypes.byref(h), 128 * 3, 128, 8, 2, 0, fake, big, None) == -1  # geometry
    assert lib.cskv_create(ctypes.byref(h), 128 * 4, 128, 8, 2, 0, ctypes.c_void_p((1 << 20) + 8), big,
                           None) == -1  # storage alignment
    assert lib.cskv_create(ctypes.byref(h), 128 * 4, 128, 8, 2, 0, fake, 100, None) == -2  # too small
    assert lib.cskv_create(ctypes.byref(h), 128 * 4, 128, 8, 2, 0, None, big, None) == -1


def test_null_table_calls():
    lib = cskv.lib()
    assert lib.cskv_workspace_bytes(None, 1, 100) == 0
    assert lib.cskv_find(None, 1, None, None, None, None, None) == -1
    assert lib.cskv_erase(None, 1, None, None, None, 0, None) == -1
    assert lib.cskv_size(None, None, None) == -1
    assert lib.cskv_clock(None) == 0
    assert lib.cskv_destroy(None) == 0
    assert lib.cskv_strerror(-2) == b"storage or workspace too small"


def test_tiered_bytes():
    """Value rows past hbm_value_rows move from device storage to host memory (Sec. 3.6)."""
    lib = cskv.lib()
    cap, dim = 128 * 64, 16
    full = lib.cskv_table_bytes(cap, 128, dim)
    assert lib.cskv_table_bytes_tiered(cap, 128, dim, cap) == full
    assert lib.cskv_host_value_bytes(cap, dim, cap) == 0
    for h in (0, 1000, cap // 2):
        dev = lib.cskv_table_bytes_tiered(cap, 128, dim, h)
        assert abs((full - dev) - (cap - h) * dim * 4) <= 256
        assert lib.cskv_host_value_bytes(cap, dim, h) == (cap - h) * dim * 4
    assert lib.cskv_table_bytes_tiered(cap, 128, dim, cap + 1) == 0
    assert lib.cskv_host_value_bytes(cap, dim, cap + 1) == 0
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)
    # a host tier without host memory, or with too little, fails before any device work
    assert lib.cskv_create_tiered(ctypes.byref(h), cap, 128, dim, 2, 0, fake, 1 << 40, 1000, None, 0, None) == -1
    assert lib.cskv_create_tiered(ctypes.byref(h), cap, 128, dim, 2, 0, fake, 1 << 40, cap + 1, None, 0, None) == -1
    assert lib.cskv_create_tiered(ctypes.byref(h), cap, 128, dim, 2, 0, fake, 1 << 40, 1000, fake, 16, None) == -2
    assert lib.cskv_row_address(None, 0) == 0
