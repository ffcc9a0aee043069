"""The C-ABI library loads on the CPU and exports every entry point that
include/phs.h declares (no compute calls: there may be no GPU)."""
import ctypes
import re
from pathlib import Path

from paper_2608_11462_amd import native as N

ROOT = Path(__file__).resolve().parents[1]


def declared():
    text = (ROOT / "include" / "phs.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert set(declared()) == set(N.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(str(N.LIB_PATH))
    for name in declared():
        assert hasattr(lib, name), name


def test_last_error_is_callable_without_a_device():
    lib = ctypes.CDLL(str(N.LIB_PATH))
    lib.phs_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.phs_last_error(), bytes)
