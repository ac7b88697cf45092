"""The C-ABI library loads and exports every entry point include/lub.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "lub.h")).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(lub_\w+)\s*\(", src, re.M)))


def test_header_lists_the_binding_names():
    from paper_1308_6482_amd import lub
    assert declared() == sorted(lub.EXPORTS)


def test_library_exports_every_symbol():
    from paper_1308_6482_amd import lub
    if not os.path.exists(lub.LIB_PATH):
        pytest.skip("liblub.so not built")
    L = ctypes.CDLL(lub.LIB_PATH)
    for name in declared():
        assert hasattr(L, name), name


def test_strerror_without_gpu():
    from paper_1308_6482_amd import lub
    if not os.path.exists(lub.LIB_PATH):
        pytest.skip("liblub.so not built")
    assert "capacity" in lub.lub_strerror(lub.LUB_ECAPACITY)
    assert lub.lub_strerror(0) == "ok"


def test_oracle_is_not_linked_into_the_product():
    """The product library and its binding never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1308_6482_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".c", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "lubref" not in txt, fn
