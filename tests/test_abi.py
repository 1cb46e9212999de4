"""The C ABI library loads and exports every entry point the header declares
(no GPU needed: nothing is called except the version string)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spx.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["spx_coo_preallocate", "spx_set_values_coo", "spx_matmult",
                 "spx_matmult_transpose", "spx_cg_solve", "spx_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2406_08646_amd import spx

    if not os.path.exists(spx.LIB_PATH):
        pytest.skip("libspx.so not built")
    lib = spx.load_library()
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(spx._SIGNATURES) == set(declared())
    assert spx.version().startswith("spx")


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2406_08646_amd import spx

    saved = spx._lib
    try:
        spx._lib = None
        with pytest.raises(RuntimeError):
            spx.load_library(str(tmp_path / "nope.so"))
    finally:
        spx._lib = saved
