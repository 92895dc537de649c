"""The C ABI library loads and exports every function include/gj.h declares.

No compute call is made here (no GPU in this tier)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gj.h")
LIB = os.path.join(ROOT, "paper_2312_00720_amd", "libgj.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gj_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gj_join", "gj_groupby", "gj_partition", "gj_last_error", "gj_version"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2312_00720_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_has_no_cpu_fallback():
    """The binding module routes every op through libgj and never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_2312_00720_amd", "__init__.py")).read()
    assert "oracle" not in src
    assert "numpy" not in src
