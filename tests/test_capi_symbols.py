"""The C-ABI library loads and exports every function include/lbm_solid.h
declares (no GPU needed: only symbol lookup and the pure host sizing call)."""
import ctypes
import os
import re

import pytest

from paper_2208_13769_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fname in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fname.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fname)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(lbm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_abi():
    names = declared_functions()
    for required in ["lbm_create", "lbm_set_material", "lbm_set_boundary", "lbm_set_fields", "lbm_step",
                     "lbm_read_fields", "lbm_workspace_bytes", "lbm_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(lbm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(lbm.EXPORTED) | set(lbm.EXPORTED_EXTRA)


def test_workspace_bytes_host_only():
    n = lbm.lbm_workspace_bytes(4096, 4096, lbm.LBM_FP32)
    # two copies of 13 float values per site plus staging and scratch
    assert 2 * 13 * 4 * 4096 * 4096 <= n <= 2 * 13 * 4 * 4096 * 4096 + (64 << 20)
    n16 = lbm.lbm_workspace_bytes(1024, 1024, lbm.LBM_FP16_STORE)
    assert 2 * (18 + 16 + 8) * 1024 * 1024 <= n16
    assert lbm.lbm_workspace_bytes(4, 100, lbm.LBM_FP64) == 0
    assert lbm.lbm_workspace_bytes(100, 100, 9) == 0


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        lbm._lib = None
        try:
            lbm.load_library(str(tmp_path / "nope.so"))
        finally:
            lbm._lib = None
