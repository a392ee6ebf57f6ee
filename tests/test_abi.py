"""CPU-side checks of the C ABI: the library loads and exports every function
include/bfs_eeds.h declares (no compute calls, no GPU needed), and the ctypes
struct layouts match the header's field lists."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfs_eeds.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(bfs_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for must in ("bfs_levels", "bfs_parents", "bfs_multi", "bfs_batch", "bfs_batch_autotune",
                 "bfs_selector_set", "bfs_mlp_forward", "bfs_mlp_loss_grad", "bfs_mlp_adam",
                 "bfs_step_time", "bfs_workspace_size", "bfs_strerror", "bfs_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2607_17106_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared_functions()) == set(_lib.SIGNATURES), "binding and header disagree"


def test_host_only_calls():
    from paper_2607_17106_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    assert lib.bfs_version() >= 1
    assert lib.bfs_strerror(-3) == b"workspace too small"
    b = ctypes.c_size_t(0)
    assert lib.bfs_workspace_size(0, 1, ctypes.byref(b)) == _lib.BFS_EINVAL
    assert lib.bfs_workspace_size(1000, 65, ctypes.byref(b)) == _lib.BFS_EINVAL


def _struct_fields(name):
    src = open(HEADER).read()
    m = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), src, flags=re.S)
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        parts = decl.replace("*", " ").split()
        type_end = 1 if parts[0] not in ("const",) else 2
        for nm in " ".join(parts[type_end:]).split(","):
            fields.append(nm.strip())
    return fields


@pytest.mark.parametrize("cname,pyname", [("bfs_graph", "BfsGraph"), ("bfs_options", "BfsOptions"),
                                          ("bfs_stats", "BfsStats"), ("bfs_graph_batch", "BfsGraphBatch"),
                                          ("bfs_batch_config", "BfsBatchConfig")])
def test_struct_layouts_match_header(cname, pyname):
    from paper_2607_17106_amd import _lib
    py = [f[0] for f in getattr(_lib, pyname)._fields_]
    assert py == _struct_fields(cname)
