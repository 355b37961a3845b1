"""The C-ABI library builds for gfx950, loads, and exports every entry point
the public header declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2501_03743_amd import sstep

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sstep.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssp_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sstep.LIB_PATH):
        from paper_2501_03743_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(sstep.LIB_PATH)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sstep.EXPORTS)


def test_status_strings_and_host_side_errors(lib):
    sstep.load()
    assert "converged" in sstep.status_string(0)
    for c in (1, 2, -1, -2, -3, -4):
        assert sstep.status_string(c)
    L = sstep.load()
    # NULL handle and bad arguments are rejected before any device work
    assert L.ssp_destroy(None) == 0
    assert L.ssp_solve(None, None, None, None, 4, 1e-8, 10, None) == sstep.EINVAL
    assert L.ssp_set_preconditioner(None, 0) == sstep.EINVAL
    assert L.ssp_get_iterations(None, None, None) == sstep.EINVAL
    assert L.ssp_last_error(None) == b""


def test_gfx950_code_object_present(lib):
    data = open(sstep.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_binding_constants_match_header():
    text = open(os.path.join(ROOT, "include", "sstep.h")).read()
    defs = dict((m.group(1), int(m.group(2)))
                for m in re.finditer(r"#define\s+(SSP_[A-Z0-9_]+)\s+(-?\d+)\b", text))
    for name, v in sstep.METHOD.items():
        assert defs["SSP_METHOD_" + name.upper()] == v, name
    for name, v in sstep.PRECISION.items():
        assert defs["SSP_PRECISION_" + name.upper()] == v, name
    assert sum(1 for k in defs if k.startswith("SSP_METHOD_")) == len(sstep.METHOD)
