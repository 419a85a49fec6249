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


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a header struct, as the C compiler lays it out."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "exactz.h"',
             "int main(void) {", '  printf("%%zu\\n", sizeof(%s));' % struct]
    for f in fields:
        lines.append('  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f))
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    return out[0], out[1:]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("cls,struct", [("Params", "exz_params"), ("Result", "exz_result"),
                                        ("Field", "exz_field")])
def test_struct_layouts(tmp_path, cls, struct):
    """The binding's ctypes structures match the header's layout exactly."""
    from paper_2604_01397_amd import exactz
    py = getattr(exactz, cls)
    names = [f[0] for f in py._fields_]
    size, offs = _c_layout(tmp_path, struct, names)
    assert ctypes.sizeof(py) == size
    assert [getattr(py, nm).offset for nm in names] == offs


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
