"""The binding's ctypes structures against include/gx.h: a small C program,
compiled with the host compiler, prints every structure's size and each
field's offset, and they must equal what ctypes lays out (a field renamed,
retyped, added or moved on one side only fails here, not in a GPU run)."""
import ctypes
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_1801_05857_amd as gx  # noqa: E402

# binding structure -> its C typedef
PAIRS = {
    "_TableOpts": "gx_table_opts",
    "_TableInfo": "gx_table_info",
    "_Stats": "gx_stats",
    "_Lts": "gx_lts",
    "_Network": "gx_network",
    "_ExploreOpts": "gx_explore_opts",
    "_ExploreResult": "gx_explore_result",
    "_Monitor": "gx_monitor",
    "_MonitoredNetwork": "gx_monitored_network",
    "_ExploreSummary": "gx_explore_summary",
    "_BatchOpts": "gx_batch_opts",
    "_TuneInfo": "gx_tune_info",
    "_ServerOpts": "gx_server_opts",
    "_ServerStats": "gx_server_stats",
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "gx.h"', "int main(void) {"]
    for py, c in PAIRS.items():
        cls = getattr(gx, py)
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for name, _ in cls._fields_:
            lines.append(f'  printf("{py} {name} %zu\\n", offsetof({c}, {name}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("layout")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                        str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    table = {}
    for line in out.splitlines():
        py, what, value = line.split()
        table[(py, what)] = int(value)
    return table


@pytest.mark.parametrize("py", sorted(PAIRS))
def test_struct_matches_header(c_layout, py):
    cls = getattr(gx, py)
    assert ctypes.sizeof(cls) == c_layout[(py, "size")]
    for name, _ in cls._fields_:
        assert getattr(cls, name).offset == c_layout[(py, name)], name
