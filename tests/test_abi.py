"""The C-ABI library loads and exports every symbol include/rbfl.h declares
(no compute calls: no GPU needed)."""
import ctypes
import os
import re

from paper_2508_04172_amd import rbfl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rbfl.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rbfl_\w+)\s*\(", text, re.M)))


def test_header_declares_binding_names():
    names = declared_functions()
    assert set(names) == set(rbfl.EXPORTED), names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(rbfl.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_layout_matches_header():
    # field order and count of rbfl_build_spec mirror the header
    text = open(os.path.join(ROOT, "include", "rbfl.h")).read()
    body = text[text.index("typedef struct {"):text.index("} rbfl_build_spec;")]
    fields = re.findall(r"\b(\w+)(?:\[[^\]]*\])*\s*;", body)
    assert fields == [f for f, _ in rbfl.BuildSpec._fields_]


def test_last_error_is_empty_string_initially():
    lib = rbfl.load()
    assert isinstance(lib.rbfl_last_error(), bytes)
