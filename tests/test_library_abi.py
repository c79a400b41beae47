"""The C-ABI library loads and exports every entry point that include/edf.h declares.
CPU only: nothing here touches a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1906_01632_amd", "libedf.so")


def declared():
    src = open(os.path.join(ROOT, "include", "edf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(edf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_calls():
    names = declared()
    for n in ("edf_create_problem", "edf_set_parameters", "edf_step", "edf_solve", "edf_moments",
              "edf_set_state", "edf_get_state", "edf_last_error", "edf_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libedf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libedf.so not built")
def test_binding_covers_the_header():
    from paper_1906_01632_amd import EXPORTS
    assert sorted(EXPORTS) == declared()


def test_library_does_not_link_the_oracle():
    """The product sources never name the oracle package."""
    for d, _, files in os.walk(os.path.join(ROOT, "paper_1906_01632_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(d, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
