"""Trained selector weights: persisting them and loading them into the library.

The weights are written by paper_2607_17106_amd.train_selector, which trains
the network with the library's own HIP forward/backward/Adam kernels on
per-level timings of the variants themselves.  Two files hold the same
values: selector_weights.bin, the binary form the C ABI's
bfs_selector_load reads (layout in include/bfs_eeds.h), and
selector_weights.npz (fp32 master parameters, feature normalisation, the
training feature range, the confidence threshold, the variant behind each of
the 4 classes, and the training metadata).  Loading goes through
bfs_selector_load.
"""
from __future__ import annotations

import os
import struct

import numpy as np

from . import _lib as L

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(_HERE, "selector_weights.bin")
NPZ_PATH = os.path.join(_HERE, "selector_weights.npz")
MAGIC = b"BFSSEL01"


def to_bytes(params, mean, std, fmin, fmax, min_conf, classes) -> bytes:
    """The bfs_selector_load file image (little-endian)."""
    params = np.asarray(params, "<f4").ravel()
    vecs = [np.asarray(x, "<f4").ravel() for x in (mean, std, fmin, fmax)]
    classes = np.asarray(classes, "<i4").ravel()
    if params.size != L.MLP_NPARAM or any(v.size != L.MLP_NFEAT for v in vecs) or classes.size != L.MLP_NCLASS:
        raise ValueError("selector arrays have the wrong sizes")
    head = MAGIC + struct.pack("<4I", 1, L.MLP_NPARAM, L.MLP_NFEAT, L.MLP_NCLASS)
    return (head + params.tobytes() + b"".join(v.tobytes() for v in vecs)
            + np.asarray([min_conf], "<f4").tobytes() + classes.tobytes())


def save(path_npz, params, mean, std, fmin, fmax, min_conf, classes, meta=None):
    """Writes the .npz and, beside it, the .bin that bfs_selector_load reads."""
    np.savez(path_npz, params=np.asarray(params, np.float32), mean=np.asarray(mean, np.float32),
             std=np.asarray(std, np.float32), fmin=np.asarray(fmin, np.float32),
             fmax=np.asarray(fmax, np.float32), min_conf=np.float32(min_conf),
             classes=np.asarray(classes, np.int32),
             meta=np.asarray(repr(meta or {})))
    with open(os.path.splitext(path_npz)[0] + ".bin", "wb") as f:
        f.write(to_bytes(params, mean, std, fmin, fmax, min_conf, classes))


def load(path: str = DEFAULT_PATH) -> bool:
    """Loads weights into the library through bfs_selector_load; False if
    the file does not exist (a malformed file raises BfsError)."""
    if path.endswith(".npz"):
        path = os.path.splitext(path)[0] + ".bin"
    if not os.path.exists(path):
        return False
    L.check(L.load().bfs_selector_load(os.fsencode(path)), "bfs_selector_load")
    return True


def load_default() -> bool:
    return load(DEFAULT_PATH)
