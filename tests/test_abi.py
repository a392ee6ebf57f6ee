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


def test_selector_file_checks_before_any_device_call(tmp_path):
    """bfs_selector_load reads and checks the whole file on the host: a
    missing, short, long or corrupted file returns BFS_EFILE (no GPU needed,
    nothing is loaded).  The shipped .bin holds exactly the shipped .npz."""
    import numpy as np
    from paper_2607_17106_amd import _lib, selector
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    with np.load(selector.NPZ_PATH, allow_pickle=False) as z:
        good = selector.to_bytes(z["params"], z["mean"], z["std"], z["fmin"], z["fmax"], float(z["min_conf"]),
                                 z["classes"])
    assert open(selector.DEFAULT_PATH, "rb").read() == good
    assert len(good) == 21244
    assert lib.bfs_selector_load(None) == _lib.BFS_EINVAL
    assert lib.bfs_selector_load(os.fsencode(str(tmp_path / "absent.bin"))) == _lib.BFS_EFILE
    nan = np.frombuffer(good, np.uint8).copy()
    nan[24:28] = np.frombuffer(np.float32(np.nan).tobytes(), np.uint8)
    bad_std = np.frombuffer(good, np.uint8).copy()
    off = 24 + 4 * (5252 + 12)  # first feature std
    bad_std[off:off + 4] = np.frombuffer(np.float32(0.0).tobytes(), np.uint8)
    bad_cls = np.frombuffer(good, np.uint8).copy()
    bad_cls[-4:] = np.frombuffer(np.int32(99).tobytes(), np.uint8)
    cases = {"short": good[:-1], "long": good + b"\0", "magic": b"BFSSEL02" + good[8:],
             "version": good[:8] + b"\2" + good[9:], "nan": nan.tobytes(), "std": bad_std.tobytes(),
             "class": bad_cls.tobytes()}
    for name, data in cases.items():
        f = tmp_path / (name + ".bin")
        f.write_bytes(data)
        assert lib.bfs_selector_load(os.fsencode(str(f))) == _lib.BFS_EFILE, name
        assert lib.bfs_selector_loaded() == 0, name
