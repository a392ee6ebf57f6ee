"""Trained selector weights: loading into the library.

The weights file (selector_weights.npz beside this module) is written by
paper_2607_17106_amd.train_selector, which trains the network with the
library's own HIP forward/backward/Adam kernels on per-level timings of the
variants themselves.  It holds the fp32 master parameters, the feature
normalisation (mean, std), the training feature range (min, max), the
confidence threshold and the variant id behind each of the 4 classes.
"""
from __future__ import annotations

import os

import numpy as np

from . import api

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.npz")


def save(path, params, mean, std, fmin, fmax, min_conf, classes, meta=None):
    np.savez(path, params=np.asarray(params, np.float32), mean=np.asarray(mean, np.float32),
             std=np.asarray(std, np.float32), fmin=np.asarray(fmin, np.float32),
             fmax=np.asarray(fmax, np.float32), min_conf=np.float32(min_conf),
             classes=np.asarray(classes, np.int32),
             meta=np.asarray(repr(meta or {})))


def load(path: str = DEFAULT_PATH) -> bool:
    """Loads weights into the library (bfs_selector_set); False if no file."""
    if not os.path.exists(path):
        return False
    with np.load(path, allow_pickle=False) as z:
        api.selector_set(z["params"], z["mean"], z["std"], z["fmin"], z["fmax"], float(z["min_conf"]),
                         z["classes"])
    return True


def load_default() -> bool:
    return load(DEFAULT_PATH)
