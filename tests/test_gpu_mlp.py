"""GPU parity of the selector network kernels and of the device-side
per-level choice, against the fp32/fp64 reference in oracle/mlp.py."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import features, heuristic, mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_17106_amd as B  # noqa: E402


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def test_forward_bit_exact_with_fp32_reference():
    rng = np.random.default_rng(0)
    p = mlp.init_params(7)
    p[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(0, .1, 64)
    p[mlp.OFF_B3:] = rng.normal(0, .1, 4)
    for B_ in (1, 63, 300):
        x = rng.standard_normal((B_, 12)).astype(np.float32) * 3
        ref, _ = mlp.forward(p, x, acc="fp32")
        got = B.mlp_forward(_dev(p), _dev(x)).cpu().numpy()
        np.testing.assert_array_equal(got, ref)


def test_predict_matches_reference():
    rng = np.random.default_rng(1)
    p = mlp.init_params(8)
    x = rng.standard_normal((500, 12)).astype(np.float32)
    cls, conf = B.mlp_predict(_dev(p), _dev(x))
    rc, rconf = mlp.predict(p, x, acc="fp32")
    np.testing.assert_array_equal(cls.cpu().numpy(), rc)
    np.testing.assert_allclose(conf.cpu().numpy(), rconf, rtol=2e-6)
    # ties go to the lowest index
    p2 = np.zeros(mlp.NPARAM, np.float32)
    p2[mlp.OFF_B3:] = [0.5, 2.0, 2.0, 2.0]
    c2, _ = B.mlp_predict(_dev(p2), _dev(np.zeros((3, 12), np.float32)))
    assert (c2.cpu().numpy() == 1).all()


def test_loss_and_gradient_against_fp64_reference():
    rng = np.random.default_rng(2)
    p = mlp.init_params(9)
    x = rng.standard_normal((256, 12)).astype(np.float32)
    y = rng.integers(0, 4, 256).astype(np.int32)
    g, loss = B.mlp_loss_grad(_dev(p), _dev(x), _dev(y, torch.int32))
    g = g.cpu().numpy().astype(np.float64)
    logits, _ = mlp.forward(p, x, acc="fp32")
    ref_g = mlp.backward(p, x, y, acc="fp32")  # straight-through at the values the fp32 forward used
    # fp32 sums over 256 rows: error bound ~ 256 * 2^-24 relative to the sum of |terms|
    scale = np.abs(ref_g).max()
    np.testing.assert_allclose(g, ref_g, rtol=1e-4, atol=2e-5 * scale)
    assert abs(float(loss.item()) - mlp.loss(logits, y)) < 1e-5 * max(1.0, mlp.loss(logits, y))


def test_adam_against_fp64_reference():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(mlp.NPARAM).astype(np.float32)
    g = rng.standard_normal(mlp.NPARAM).astype(np.float32)
    m = rng.standard_normal(mlp.NPARAM).astype(np.float32) * .1
    v = np.abs(rng.standard_normal(mlp.NPARAM)).astype(np.float32) * .01
    dp, dm, dv = _dev(p), _dev(m), _dev(v)
    B.mlp_adam(dp, _dev(g), dm, dv, 5, 1e-3)
    rp, rm, rv = mlp.adam(p, g, m, v, 5, 1e-3)
    # The kernel works in fp32 with fp32 constants: 0.9f and 0.999f differ from
    # 0.9 and 0.999 by up to 2.4e-8 and 5e-8 (relative 1 - beta errors 2.4e-7
    # and 5e-5), plus one rounding per operation (2^-24 relative).
    g64, m64, v64 = (a.astype(np.float64) for a in (g, m, v))
    bm = 2.5e-7 * np.abs(g64) + 3e-8 * np.abs(m64) + 2 * 2.0 ** -24 * (np.abs(rm) + np.abs(g64))
    bv = 6e-5 * g64 * g64 + 6e-8 * np.abs(v64) + 2 * 2.0 ** -24 * (np.abs(rv) + g64 * g64)
    assert (np.abs(dm.cpu().numpy() - rm) <= bm).all()
    assert (np.abs(dv.cpu().numpy() - rv) <= bv).all()
    # update: lr * mhat / (sqrt(vhat) + eps) with the above relative errors
    np.testing.assert_allclose(dp.cpu().numpy(), rp, rtol=0, atol=3e-7 * (1 + np.abs(rp)).max())


def test_gpu_training_learns_a_teacher():
    """Labels from a fixed random teacher network (oracle forward); the GPU
    kernels (forward, gradient, Adam) must fit them."""
    rng = np.random.default_rng(4)
    teacher = mlp.init_params(100) * 2
    x = rng.standard_normal((2048, 12)).astype(np.float32)
    y, _ = mlp.predict(teacher, x)
    p = _dev(mlp.init_params(5))
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    dx, dy = _dev(x), _dev(y.astype(np.int32), torch.int32)
    losses = []
    for step in range(1, 301):
        g, loss = B.mlp_loss_grad(p, dx, dy)
        B.mlp_adam(p, g, m, v, step, 3e-3)
        losses.append(float(loss.item()))
    acc = (B.mlp_predict(p, dx)[0].cpu().numpy() == y).mean()
    assert losses[-1] < 0.5 * losses[0]
    assert acc > 0.8


def _selector_case(g, s, params, mean, std, fmin, fmax, min_conf, classes):
    """Expected per-level variants of the learned mode, from the oracle's
    depths and features."""
    ref, _, nl = oracle.bfs(g.row_ptr, g.col_idx, int(s))
    feats = features.level_features(g.row_ptr, g.csc_ptr, ref)
    prof = oracle.level_profile(g.row_ptr, g.csc_ptr, g.csc_idx, ref)
    dirs = heuristic.replay(g.n, prof["nF"], prof["eF"], prof["eU"])
    xn = ((feats - mean.astype(np.float32)) / std.astype(np.float32)).astype(np.float32)
    cls, conf = mlp.predict(params, xn, acc="fp32")
    conf32 = conf.astype(np.float32)
    oor = ((feats < fmin) | (feats > fmax)).any(axis=1)
    fb = oor | ~(conf32 >= np.float32(min_conf))
    heur = np.where(np.array(dirs) == 1, B.PULL_B, B.PUSH_Q_BLOCK)
    exp = np.where(fb, heur, np.asarray(classes)[cls])
    return ref, exp, fb


@pytest.mark.parametrize("loop_flag", [0, "device"])
def test_device_decisions_match_reference(loop_flag):
    flags = B.F_DEVICE_LOOP if loop_flag == "device" else 0
    g = gg.rmat(15, seed=4015).with_csc()
    dg = B.DeviceGraph.from_graph(g)
    rng = np.random.default_rng(6)
    params = mlp.init_params(11)
    params[mlp.OFF_B3:] = rng.normal(0, 1, 4)
    mean = rng.normal(0, 1, 12).astype(np.float32)
    std = (0.5 + rng.random(12)).astype(np.float32)
    classes = [B.PUSH_Q_BLOCK, B.PUSH_Q_MERGE, B.PUSH_B_NOATOMIC, B.PULL_B]
    wide_min, wide_max = np.full(12, -1e30, np.float32), np.full(12, 1e30, np.float32)
    try:
        for min_conf, fmin, fmax in ((0.0, wide_min, wide_max), (0.45, wide_min, wide_max),
                                     (0.0, wide_min, np.full(12, 3.0, np.float32)), (1.01, wide_min, wide_max)):
            B.selector_set(params, mean, std, fmin, fmax, min_conf, classes)
            for s in gg.pick_sources(g, 3, 12):
                ref, exp, fb = _selector_case(g, s, params, mean, std, fmin, fmax, min_conf, classes)
                lv, par, st = B.bfs_parents(dg, int(s), variant=B.AUTO_LEARNED, level_stats=True, flags=flags)
                np.testing.assert_array_equal(lv.cpu().numpy(), ref)
                np.testing.assert_array_equal(st["variant"], exp)
                np.testing.assert_array_equal(st["fallback"].astype(bool), fb)
                assert st["fell_back"] == int(fb.any())
    finally:
        B.selector_clear()


def test_level_features_match_reference():
    for g in (gg.workload("rmat14").with_csc(), gg.directed_random(3000, 20000, seed=8)):
        dg = B.DeviceGraph.from_graph(g)
        for s in gg.pick_sources(g, 3, 3):
            lv, st = B.bfs_levels(dg, int(s), variant=B.AUTO_HEURISTIC, level_stats=True)
            f = B.level_features(st, g.n, g.nnz)
            ref = features.level_features(g.row_ptr, g.csc_ptr, lv.cpu().numpy())
            np.testing.assert_array_equal(f, ref)


def test_graph_sums_and_given_sums_path():
    """bfs_graph_sums equals the sums written out from the degrees, and a
    learned search fed those sums (BFS_F_GRAPH_SUMS, what the binding does)
    chooses exactly as one that computes them itself (raw C call without the
    flag)."""
    import ctypes
    from paper_2607_17106_amd import _lib as L, api
    g = gg.rmat(15, seed=4015).with_csc()
    dg = B.DeviceGraph.from_graph(g)
    ld = np.floor(np.log2(1 + np.diff(g.row_ptr).astype(np.float64))).astype(np.int64)
    assert dg.graph_sums() == (int(ld.sum()), int((ld * ld).sum()))
    rng = np.random.default_rng(16)
    params = mlp.init_params(21)
    params[mlp.OFF_B3:] = rng.normal(0, 1, 4)
    wide_min, wide_max = np.full(12, -1e30, np.float32), np.full(12, 1e30, np.float32)
    classes = [B.PUSH_Q_BLOCK, B.PUSH_Q_MERGE, B.PUSH_B_NOATOMIC, B.PULL_B]
    try:
        B.selector_set(params, np.zeros(12, np.float32), np.ones(12, np.float32), wide_min, wide_max, 0.0, classes)
        for s in gg.pick_sources(g, 3, 17):
            lv1, st1 = B.bfs_levels(dg, int(s), variant=B.AUTO_LEARNED, level_stats=True)
            opt, _ = api._options(B.AUTO_LEARNED, L.F_LEVEL_STATS, None, None, 0, None)
            sb = api._StatsBuf(4096)
            lv2 = torch.empty(g.n, dtype=torch.int32, device="cuda")
            L.check(L.load().bfs_levels(dg.c, int(s), api._ptr(lv2), ctypes.byref(opt), ctypes.byref(sb.s),
                                        api._stream(None)), "bfs_levels")
            st2 = sb.as_dict(True)
            assert not (opt.flags & L.F_GRAPH_SUMS)
            np.testing.assert_array_equal(st1["variant"], st2["variant"])
            np.testing.assert_array_equal(lv1.cpu().numpy(), lv2.cpu().numpy())
            assert (st1["graph_ld"], st1["graph_ld2"]) == (st2["graph_ld"], st2["graph_ld2"]) == dg.graph_sums()
    finally:
        B.selector_clear()
