"""The HIP library loads and exports every symbol include/exactz.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2604_01397_amd", "libexactz.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "exactz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(exz_[a-z_]+)\s*\(", src)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_match_header():
    from paper_2604_01397_amd import exactz
    assert sorted(exactz.EXPORTS) == _declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_struct_layouts():
    from paper_2604_01397_amd import exactz
    assert ctypes.sizeof(exactz.Params) == 64
    assert ctypes.sizeof(exactz.Result) == 104
    assert ctypes.sizeof(exactz.Field) == 64 + 32


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings_and_workspace_without_gpu():
    from paper_2604_01397_amd import exactz
    lib = exactz.load()
    assert lib.exz_status_string(0) == b"ok"
    assert lib.exz_status_string(-3).startswith(b"decompressed")
    # workspace sizing is host arithmetic: no device needed
    small = exactz.workspace_bytes((64, 64))
    big = exactz.workspace_bytes((512, 512, 512))
    assert 0 < small < big
    assert exactz.workspace_bytes((0, 5)) == 0
    # ~ (1 + 4 + 1 + 1/8 + ...) bytes per vertex plus worst-case CP arrays
    assert 30 * 512 ** 3 < big < 60 * 512 ** 3
