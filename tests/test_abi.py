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
