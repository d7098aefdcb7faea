"""include/tw.h compiles as plain C11, and the structure layouts the ctypes
binding declares are the ones a C compiler gives the header.  A C program
linked with libtw.so also runs the host-only entry points (no device call).
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1709_09990_amd import tw as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def c_program(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    if not os.path.exists(T.LIB_PATH):
        pytest.fail("libtw.so is not built")
    exe = str(tmp_path_factory.mktemp("cabi") / "abi_check")
    lib_dir = os.path.dirname(T.LIB_PATH)
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-pedantic",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_check.c"),
           "-L", lib_dir, "-ltw", "-Wl,-rpath," + lib_dir, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=60).stdout
    fields = {}
    for line in out.splitlines():
        parts = line.split()
        fields[parts[0]] = parts[1:]
    return fields


def test_struct_layouts_match_binding(c_program):
    f = c_program
    assert int(f["sizeof_options"][0]) == ctypes.sizeof(T._Options)
    for name in ("mmw_prune", "reductions", "batch_schedule", "batch_chunk", "workspace", "workspace_bytes",
                 "fault_inject_level", "capture"):
        assert int(f["off_" + name][0]) == getattr(T._Options, name).offset, name
    assert int(f["sizeof_stats"][0]) == ctypes.sizeof(T._Stats)
    assert int(f["sizeof_graph_stats"][0]) == ctypes.sizeof(T._GraphStats)
    assert int(f["sizeof_level_record"][0]) == ctypes.sizeof(T._LevelRecord)
    assert int(f["sizeof_graph"][0]) == ctypes.sizeof(T._Graph)
    assert int(f["sizeof_batch_level"][0]) == ctypes.sizeof(T._BatchLevel)


def test_host_entry_points_from_c(c_program):
    # 5-cycle: minor-min-width 2, the identity order has width 2, its tree
    # decomposition width 2, a maximum clique is an edge
    assert c_program["mmw"] == ["2", "width", "2", "decomposition_width", "2", "clique_bits", "2"]
    assert c_program["status_str"]
