"""The wave-level scan steps the kernels run on DPP moves (common.hpp
wave_incl_scan / wave_sum_u64 / wave_or_u64 / wave_max_nonneg, and the
segmented OR of msbfs.hip's ms_seg_or), replayed on the host with the moves'
documented lane semantics: row_shr:k gives lane l the value of lane l-k of
its 16-lane row (no source for the row's first k lanes), row_bcast:15 gives
every lane of rows 1 and 3 (row mask 0xa) the last lane of the row before,
row_bcast:31 gives rows 2 and 3 (row mask 0xc) lane 31, and a lane with no
source keeps the move's old value.  The GPU tests run the real moves; this
pins the step sequence itself: it must produce an inclusive scan for any
input, and the segmented OR must equal the plain definition for keys that do
not decrease (with trailing -1 keys), so a wrong shift, row mask or key test
fails here."""
import numpy as np

W = 64


def move(x, ctrl, rows, old):
    out = np.array(old, dtype=object)
    for l in range(W):
        r = l // 16
        if not (rows >> r) & 1:
            continue
        if ctrl[0] == "shr":
            k = ctrl[1]
            if l % 16 >= k:
                out[l] = x[l - k]
        elif ctrl == ("bcast", 15):
            if r >= 1:
                out[l] = x[16 * r - 1]
        elif ctrl == ("bcast", 31):
            if r >= 2:
                out[l] = x[31]
    return out


STEPS = [(("shr", 1), 0xF), (("shr", 2), 0xF), (("shr", 4), 0xF), (("shr", 8), 0xF),
         (("bcast", 15), 0xA), (("bcast", 31), 0xC)]


def dpp_scan(x, op, identity):
    x = np.array(x, dtype=object)
    for ctrl, rows in STEPS:
        y = move(x, ctrl, rows, [identity] * W)
        x = np.array([op(a, b) for a, b in zip(x, y)], dtype=object)
    return x


def dpp_seg_or(x, key):
    x = np.array(x, dtype=object)
    key = np.array(key, dtype=object)
    for ctrl, rows in STEPS:
        yk = move(key, ctrl, rows, [~k for k in key])
        yx = move(x, ctrl, rows, [0] * W)
        x = np.array([a | b if yk[i] == key[i] else a for i, (a, b) in enumerate(zip(x, yx))], dtype=object)
    nxt = [key[l + 1] if l + 1 < W else ~key[l] for l in range(W)]  # wave_shl:1
    tail = [nxt[l] != key[l] for l in range(W)]
    return x, tail


def test_inclusive_scans():
    rng = np.random.default_rng(7)
    for _ in range(50):
        x = [int(v) for v in rng.integers(0, 1 << 40, W)]
        got = dpp_scan(x, lambda a, b: a + b, 0)
        assert list(got) == list(np.cumsum(np.array(x, dtype=object)))
        assert got[W - 1] == sum(x)  # the lane the wave sum reads
        m = [int(v) for v in rng.integers(0, 1 << 20, W)]
        assert dpp_scan(m, max, 0)[W - 1] == max(m)
        o = [int(v) for v in rng.integers(0, 1 << 62, W)]
        acc = 0
        for v in o:
            acc |= v
        assert dpp_scan(o, lambda a, b: a | b, 0)[W - 1] == acc


def test_segmented_or_matches_definition():
    rng = np.random.default_rng(11)
    for trial in range(200):
        cuts = np.sort(rng.choice(np.arange(1, W), size=rng.integers(0, 20), replace=False))
        key = np.zeros(W, dtype=np.int64)
        for c in cuts:
            key[c:] += 1
        key += int(rng.integers(0, 5))
        tail_end = int(rng.integers(0, 8)) if trial % 2 else 0  # lanes past the end: key -1, value 0
        x = [int(v) for v in rng.integers(0, 1 << 62, W)]
        if tail_end:
            key[W - tail_end:] = -1
            for l in range(W - tail_end, W):
                x[l] = 0
        key = [int(k) for k in key]
        got, tail = dpp_seg_or(x, key)
        for l in range(W):
            want = 0
            for j in range(l, -1, -1):
                if key[j] != key[l]:
                    break
                want |= x[j]
            assert got[l] == want, (trial, l)
            assert tail[l] == (l == W - 1 or key[l + 1] != key[l])
