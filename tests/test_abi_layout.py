"""The Python binding's structures have the layout include/kairos.h gives
them: a C program compiled against the header reports every structure's
size and every field's offset, and the ctypes declarations must agree."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ("kairos_index_view", "kairos_tuning", "kairos_profile", "kairos_server_opts", "kairos_completion",
           "kairos_server_stats")


@pytest.fixture(scope="module")
def binding():
    return pytest.importorskip("paper_2401_02563_amd")


def c_layout(tmp_path, binding):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "kairos.h"', "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, *_ in getattr(binding, name)._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        parts = line.split()
        got[tuple(parts[:-1])] = int(parts[-1])
    return got


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_binding_structures_match_the_header(tmp_path, binding):
    import ctypes
    got = c_layout(tmp_path, binding)
    for name in STRUCTS:
        cls = getattr(binding, name)
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, *_ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
