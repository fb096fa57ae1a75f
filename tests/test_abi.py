"""The C-ABI library loads and exports every symbol include/am.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "am.h")
LIB = os.path.join(ROOT, "paper_2106_10031_amd", "libam.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(am_[a-z_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared()
    for n in ["am_create", "am_destroy", "am_load_net", "am_seed_rays", "am_march", "am_fetch"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libam.so not built")
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_lists_every_declared_symbol():
    from paper_2106_10031_amd import binding
    assert sorted(binding.EXPORTS) == declared()


def test_library_has_no_oracle_dependency():
    # the product library must not link or name the CPU reference
    if not os.path.exists(LIB):
        pytest.skip("libam.so not built")
    data = open(LIB, "rb").read()
    assert b"orc_" not in data and b"am_oracle" not in data
