"""The C-ABI library loads and exports every symbol include/rbfl.h declares
(no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

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


def test_variant_counts_without_a_device():
    """rbfl_variants is host-only: a count per tunable form, a negative code
    (raised as ValueError by the binding) for the surrogate form."""
    assert rbfl.variants(rbfl.FORM_FP64) >= 2
    assert rbfl.variants(rbfl.FORM_FP32) >= 1 and rbfl.variants(rbfl.FORM_BF16) >= 1
    assert rbfl.variants(rbfl.FORM_SPLIT) == 4          # digit counts S = 5..8
    assert rbfl.load().rbfl_variants(rbfl.FORM_SURROGATE) < 0
    with pytest.raises(ValueError):
        rbfl.variants(rbfl.FORM_SURROGATE)
