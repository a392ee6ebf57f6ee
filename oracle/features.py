"""Per-level selector features from exact BFS depths -- TEST INFRASTRUCTURE ONLY.

The selector's 12 inputs for level k, with F_k = {depth = k},
P_k = {0 <= depth <= k}, U_k = V minus P_k, and ld(v) = floor(log2(1 + outdeg v)):
  0 log2(1+|F_k|)  1 log2(1+eF)  2 log2(1+|U_k|)  3 log2(1+eU)
  4 |F_k|/n  5 eF/nnz  6 |U_k|/n  7 mean ld over F_k  8 variance of ld over F_k
  9 mean ld over V  10 variance of ld over V  11 log2(1+k)
where eF sums out-degrees over F_k and eU sums in-degrees over U_k.  Every
sum is an exact integer; the arithmetic on them is fp64, rounded to fp32 at
the end (the selector's definition).  Vertices with no in-edges count as
unvisited here exactly as everywhere else (U_k is defined by the depths).
"""
from __future__ import annotations

import numpy as np


def level_features(row_ptr, csc_ptr, levels) -> np.ndarray:
    rp = np.asarray(row_ptr, dtype=np.int64)
    cp = np.asarray(csc_ptr, dtype=np.int64)
    lv = np.asarray(levels)
    n = lv.shape[0]
    nnz = int(rp[-1])
    od = np.diff(rp)
    idg = np.diff(cp)
    # floor(log2(1+d)) exactly: 1+d = m * 2^e with m in [0.5, 1) gives e-1
    ld = (np.frexp((1 + od).astype(np.float64))[1] - 1).astype(np.int64)
    gld, gld2 = int(ld.sum()), int((ld * ld).sum())
    nl = int(lv.max()) + 1 if (lv >= 0).any() else 0
    out = np.zeros((nl, 12), dtype=np.float32)
    reached = 0
    in_reached = 0
    for k in range(nl):
        F = lv == k
        nF = int(F.sum())
        reached += nF
        in_reached += int(idg[F].sum())
        eF = int(od[F].sum())
        nU = n - reached
        eU = nnz - in_reached
        fld, fld2 = int(ld[F].sum()), int((ld[F] ** 2).sum())
        fm = fld / nF if nF else 0.0
        f = [np.log2(1.0 + nF), np.log2(1.0 + eF), np.log2(1.0 + nU), np.log2(1.0 + eU),
             nF / n, eF / nnz if nnz else 0.0, nU / n, fm, (fld2 / nF - fm * fm) if nF else 0.0,
             gld / n, gld2 / n - (gld / n) ** 2, np.log2(1.0 + k)]
        out[k] = np.array(f, dtype=np.float64).astype(np.float32)
    return out
