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


def _struct_fields(name):
    """(type, name, count) of the fields of `typedef struct { ... } name;` in the header."""
    src = open(os.path.join(ROOT, "include", "edf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", src).group(1)
    out = []
    for t, names in re.findall(r"(int32_t|double)\s+([^;]+);", body):
        for d in names.split(","):
            n, cnt = re.fullmatch(r"\s*(\w+)\s*(?:\[(\d+)\])?\s*", d).groups()
            out.append((t, n, int(cnt) if cnt else None))  # None: not an array
    return out


@pytest.mark.parametrize("header_name,binding_name", [
    ("edf_group_desc", "GroupDesc"), ("edf_physics", "PhysicsC"),
    ("edf_solver_opts", "SolverOpts"), ("edf_step_stats", "StepStats")])
def test_binding_structs_match_the_header(header_name, binding_name):
    """The ctypes structure has the header's fields, in order, with the same types, so the
    options reach the library as declared."""
    from paper_1906_01632_amd import _binding
    ct = {"int32_t": ctypes.c_int32, "double": ctypes.c_double}
    want = _struct_fields(header_name)
    got = getattr(_binding, binding_name)._fields_
    assert [n for _, n, _ in want] == [n for n, _ in got]
    for (t, n, cnt), (_, bt) in zip(want, got):
        if cnt is None:
            assert bt is ct[t], n
        else:
            assert issubclass(bt, ctypes.Array) and bt._type_ is ct[t] and bt._length_ == cnt, n
