"""Pins of the selector-network reference and the direction-rule replay.

* bf16 rounding against torch's own float32 -> bfloat16 conversion (an
  independent implementation of round-to-nearest-even) and hand-picked ties;
* a hand-derived forward pass (tests/golden/mlp_hand_example.json);
* fp32 accumulation against fp64 within the fp32 rounding bound;
* the backward pass against central finite differences in fp64;
* the first Adam step against its closed form (lr * sign(g) up to eps);
* the direction rule on hand-made count sequences.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import mlp, heuristic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 20000),
                        np.array([0.0, -0.0, 1.0, 65504.0, 3.4e38, -3.4e38, 1e-40, np.inf, -np.inf],
                                 dtype=np.float32)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)


def test_bf16_round_ties_to_even():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    x = np.array([one + ulp / 2, one + 3 * ulp / 2, one + ulp / 2 + np.float32(2 ** -20)], dtype=np.float32)
    np.testing.assert_array_equal(mlp.bf16_round(x), np.array([1.0, 1.0 + 2 * ulp, 1.0 + ulp], np.float32))


def _hand_params():
    gd = json.load(open(os.path.join(GOLD, "mlp_hand_example.json")))
    p = np.zeros(mlp.NPARAM, np.float32)
    W1 = p[mlp.OFF_W1:mlp.OFF_B1].reshape(64, 12)
    W2 = p[mlp.OFF_W2:mlp.OFF_B2].reshape(64, 64)
    W3 = p[mlp.OFF_W3:mlp.OFF_B3].reshape(4, 64)
    for i, j, v in gd["W1_nonzero"]:
        W1[i, j] = v
    for i, j, v in gd["W2_nonzero"]:
        W2[i, j] = v
    for i, j, v in gd["W3_nonzero"]:
        W3[i, j] = v
    for i, v in gd["b1_nonzero"]:
        p[mlp.OFF_B1 + i] = v
    for i, v in gd["b2_nonzero"]:
        p[mlp.OFF_B2 + i] = v
    for i, v in gd["b3_nonzero"]:
        p[mlp.OFF_B3 + i] = v
    return p, gd


@pytest.mark.parametrize("acc", ["fp32", "fp64"])
def test_forward_hand_example(acc):
    p, gd = _hand_params()
    x = np.array([gd["x"]], np.float32)
    logits, _ = mlp.forward(p, x, acc=acc)
    np.testing.assert_array_equal(logits[0], np.array(gd["logits"]))
    l = mlp.loss(logits, [gd["label"]])
    assert abs(l - (math.log(math.exp(7) + math.exp(3.5) + math.exp(-7) + math.exp(0.25)) - 3.5)) < 1e-12


def test_fp32_accumulation_within_rounding_bound():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3)
    x = rng.standard_normal((256, 12)).astype(np.float32)
    # first layer only: both modes see identical bf16 inputs and weights
    W1, b1 = mlp.unpack(p)[:2]
    h0 = mlp.bf16_round(x)
    W1r = mlp.bf16_round(W1)
    z32 = mlp._layer(h0, W1r, b1, "fp32").astype(np.float64)
    z64 = mlp._layer(h0, W1r, b1, "fp64")
    bound = 13 * 2.0 ** -24 * (np.abs(h0).astype(np.float64) @ np.abs(W1r.astype(np.float64)).T + np.abs(b1))
    assert (np.abs(z32 - z64) <= bound + 1e-30).all()
    # whole network with rounding switched off: fp32 close to fp64
    l32, _ = mlp.forward(p, x, acc="fp32", rounding=False)
    l64, _ = mlp.forward(p, x, acc="fp64", rounding=False)
    np.testing.assert_allclose(l32, l64, rtol=1e-5, atol=1e-5)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = mlp.init_params(4).astype(np.float64)
    x = rng.standard_normal((16, 12))
    y = rng.integers(0, 4, 16)
    g = mlp.backward(p, x, y, acc="fp64", rounding=False)
    f = lambda q: mlp.loss(mlp.forward(q, x, acc="fp64", rounding=False)[0], y)
    idx = np.concatenate([rng.choice(np.arange(mlp.OFF_W1, mlp.OFF_B1), 30, replace=False),
                          np.arange(mlp.OFF_B1, mlp.OFF_B1 + 10),
                          rng.choice(np.arange(mlp.OFF_W2, mlp.OFF_B2), 40, replace=False),
                          np.arange(mlp.OFF_B2, mlp.OFF_B2 + 10),
                          np.arange(mlp.OFF_W3, mlp.NPARAM)])
    h = 1e-6
    for i in idx:
        qp = p.copy(); qp[i] += h
        qm = p.copy(); qm[i] -= h
        fd = (f(qp) - f(qm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_backward_uses_rounded_values():
    # with rounding on, the gradient is the straight-through one evaluated at
    # the bf16 values: equal to the no-rounding gradient at pre-rounded inputs
    # when every weight and input is already a bf16 value and activations stay
    # bf16-exact (hand example).
    p, gd = _hand_params()
    x = np.array([gd["x"]], np.float32)
    g1 = mlp.backward(p, x, [gd["label"]], acc="fp64", rounding=True)
    g2 = mlp.backward(p.astype(np.float64), x.astype(np.float64), [gd["label"]], acc="fp64", rounding=False)
    np.testing.assert_allclose(g1, g2, rtol=0, atol=1e-15)
    # closed form for the output bias: softmax - onehot
    z = np.array(gd["logits"])
    sm = np.exp(z - z.max()) / np.exp(z - z.max()).sum()
    sm[gd["label"]] -= 1
    np.testing.assert_allclose(g1[mlp.OFF_B3:], sm, rtol=1e-12)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    lr = 0.01
    p1, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), 1, lr)
    exp = p - lr * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p1, exp, rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_predict_ties_to_lowest_index():
    p = np.zeros(mlp.NPARAM, np.float32)
    p[mlp.OFF_B3:] = [1.0, 2.0, 2.0, 0.0]
    cls, conf = mlp.predict(p, np.zeros((3, 12), np.float32))
    assert (cls == 1).all()


def test_direction_rule_replay():
    n = 2400
    # level 0: tiny frontier -> push; level 1: frontier edges exceed unvisited
    # edges / 14 -> pull; level 2: frontier still growing -> stay pull;
    # level 3: shrinking and below n/24 -> push.
    nF = [1, 50, 900, 60, 10]
    eF = [10, 1500, 20000, 300, 40]
    eU = [20000, 19990, 9000, 500, 1000]
    assert heuristic.replay(n, nF, eF, eU) == [0, 1, 1, 0, 0]
    # never switches when the frontier stays light
    assert heuristic.replay(n, [1, 2, 3], [1, 2, 3], [10 ** 6] * 3) == [0, 0, 0]
    # boundary: eF * 14 == eU stays push (strict inequality)
    assert heuristic.replay(n, [1], [100], [1400]) == [0]
    assert heuristic.replay(n, [1], [101], [1400]) == [1]
