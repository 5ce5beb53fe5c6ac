"""Host-side checks of the C ABI: the library loads and exports every entry point
include/gpe.h declares (no compute calls; CPU only)."""
import ctypes
import os
import re

from paper_2404_14401_amd import gpe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gpe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gpe_[a-z_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert declared() == sorted(gpe.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(gpe.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_message_is_empty_string_initially():
    assert isinstance(gpe.lib().gpe_last_error(), bytes)
