"""The C-ABI library loads and exports every entry point include/tomo.h declares."""

import os
import re

import paper_2003_12677_amd as tomo

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tomo.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:tomo_status|void|const char\*)\s+(tomo_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tomo_build_operator", "tomo_project", "tomo_backproject", "tomo_solve",
                     "tomo_destroy_operator"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = tomo.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(tomo.SIGNATURES)


def test_version_and_error_string():
    lib = tomo.load()
    assert tomo.version() == "1.0.0"
    assert isinstance(lib.tomo_last_error(), bytes)


def test_documented_tuning_defaults_and_field_order_match_the_library():
    """The header states the tuning defaults in field order; the binding's struct mirrors the
    header's field order."""
    text = open(HEADER).read()
    m = re.search(r"Defaults \(in field order\):\s*([0-9,\s]+)\.", text)
    assert m, "defaults line missing"
    documented = [int(v) for v in m.group(1).replace("\n", " ").split(",")]
    body = text[text.index("typedef struct {", text.index("Kernel layout parameters")):]
    body = body[:body.index("} tomo_tuning;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"int32_t\s+(\w+);", body)
    op = tomo.Operator(8, 6, 9, device=-1)
    tuning = op.get_tuning()
    op.close()
    assert fields == list(tuning.keys())
    assert documented == list(tuning.values())
