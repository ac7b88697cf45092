"""The binding's ctypes structures against the C header: every field of
every public struct at the same offset, every struct of the same size, as
gcc lays them out from include/lub.h (no GPU needed)."""
import ctypes as C
import os
import subprocess

import pytest

from paper_1308_6482_amd import lub as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["lub_params_t", "lub_domain_t", "lub_opts_t", "lub_stats_t", "lub_step_t",
           "lub_grow_t", "lub_train_cfg_t"]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    """{struct: (size, {field: offset})} printed by a program compiled
    against the header."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lub.h"', 'int main(void) {']
    for name in STRUCTS:
        cls = getattr(L, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ['  return 0;', '}']
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for ln in out.splitlines():
        name, field, val = ln.split()
        size, fields = res.setdefault(name, [None, {}])
        if field == "size":
            res[name][0] = int(val)
        else:
            fields[field] = int(val)
    return res


@pytest.mark.parametrize("name", STRUCTS)
def test_struct_matches_header(c_layout, name):
    cls = getattr(L, name)
    size, fields = c_layout[name]
    assert C.sizeof(cls) == size, name
    for field, _ in cls._fields_:
        assert getattr(cls, field).offset == fields[field], f"{name}.{field}"
