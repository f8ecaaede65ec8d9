"""Pins for the CPU reference of the frontier predictor: central finite
differences of its own loss, closed-form special cases, bfloat16 rounding."""

import math

import numpy as np
import pytest

from oracle import mlp_ref as M


def batch(rng, n, n_sym):
    sym = rng.integers(0, n_sym, n)
    arity = rng.integers(0, 4, n)
    bits = rng.integers(0, 32, n)
    bucket = rng.integers(0, 16, n)
    label = rng.integers(0, 2, n)
    return sym, arity, bits, bucket, label


def test_bf16_rounding():
    # values exactly representable stay; ties go to even; known roundings
    assert M.bf16_round([1.0, -2.5, 0.0])[0] == 1.0
    assert M.bf16_round([1.0 + 2 ** -8])[0] == 1.0            # tie -> even (1.0)
    assert M.bf16_round([1.0 + 3 * 2 ** -8])[0] == 1.0 + 2 ** -6  # tie -> even
    assert M.bf16_round([1.0 + 2 ** -7])[0] == 1.0 + 2 ** -7
    x = np.random.default_rng(0).normal(size=1000)
    r = M.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8 + 1e-30)
    assert np.array_equal(M.bf16_round(r), r)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradients_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    n_sym = 7
    params = M.init_params(n_sym, seed)
    # move biases off zero so that no ReLU sits exactly at its kink
    params["b1"] = rng.normal(0, 0.3, params["b1"].shape)
    params["b2"] = rng.normal(0, 0.3, params["b2"].shape)
    data = batch(rng, 40, n_sym)
    loss, p, g = M.forward_backward(params, *data)
    flat = M.flatten(params)
    gflat = M.flatten(g)
    idx = rng.choice(len(flat), size=80, replace=False)
    h = 1e-6
    for i in idx:
        up, dn = flat.copy(), flat.copy()
        up[i] += h
        dn[i] -= h
        num = (M.loss_only(M.unflatten(up, n_sym), *data) -
               M.loss_only(M.unflatten(dn, n_sym), *data)) / (2 * h)
        assert abs(num - gflat[i]) <= 1e-6 + 1e-5 * abs(num), (i, num, gflat[i])


def test_output_bias_gradient_closed_form():
    # d loss / d b3 = mean(p - y)
    rng = np.random.default_rng(5)
    params = M.init_params(4, 5)
    data = batch(rng, 64, 4)
    loss, p, g = M.forward_backward(params, *data)
    assert g["b3"][0] == pytest.approx(np.mean(p - data[4]), rel=1e-12, abs=1e-15)


def test_zero_network_predicts_half():
    # all-zero weights: z = 0, p = 1/2, loss = log 2 whatever the labels
    n_sym = 3
    params = {k: np.zeros(s) for k, s in M.param_shapes(n_sym).items()}
    data = batch(np.random.default_rng(1), 10, n_sym)
    loss, p, g = M.forward_backward(params, *data)
    assert np.allclose(p, 0.5)
    assert loss == pytest.approx(np.log(2.0))
    assert np.all(g["W1"] == 0) and np.all(g["E"] == 0)


def test_feature_layout():
    E = np.arange(2 * 16, dtype=np.float64).reshape(2, 16)
    x = M.features(E, [1], [3], [0b10110], [15])
    assert np.array_equal(x[0, :16], E[1])
    assert x[0, 16] == 3 / 8
    assert list(x[0, 17:22]) == [0, 1, 1, 0, 1]
    assert x[0, 22] == 1.0 and x[0, 23] == 0.0


def test_age_bucket():
    # bucket(0)=0, then floor(log2 a)+1 capped at 15
    a = np.array([0, 1, 2, 3, 4, 7, 8, 1023, 1024, 8191, 8192, 16383, 16384, 10 ** 9])
    assert list(M.age_bucket(a)) == [0, 1, 2, 2, 3, 3, 4, 10, 11, 13, 14, 14, 15, 15]


def test_record_round_trip():
    rng = np.random.default_rng(3)
    f = batch(rng, 100, 4096)
    rec = M.encode_records(*f)
    for a, b in zip(f, M.decode_records(rec)):
        assert np.array_equal(np.asarray(a), b)
    # field positions (spot check)
    assert int(M.encode_records([5], [2], [0b11], [4], [1])[0]) == (5 | 2 << 16 | 3 << 20 | 4 << 25 | 1 << 32)


def test_decision_table_matches_forward():
    params = M.init_params(3, 9)
    tab = M.decision_table(params, 3, [0, 1, 2], 0.1)
    assert tab.shape == (3, 32, 16)
    sym, bits, bucket = 2, 0b10101, 7
    p = M.forward_backward(params, [sym], [2], [bits], [bucket], [0])[1][0]
    assert tab[sym, bits, bucket] == pytest.approx(p, rel=1e-12)


def test_forward_values_computed_by_hand():
    """A two-symbol network with a few non-zero weights, evaluated by hand.

    Record A: symbol 0 (E = [0.5, -1, 0...]), arity 2, argument bits 0b00101,
    age bucket 3, label 1.  Record B: symbol 1 (E = [0, 0, 1.5, 0...]),
    arity 1, bits 0b11110, bucket 0, label 0.  Inputs: x16 = arity/8,
    x17..x21 = c_0..c_4, x22 = bucket/15.

        h1_0 = relu(2 x0)                      A: 1      B: 0
        h1_1 = relu(x1 + 0.5)                  A: 0      B: 0.5   (A: -0.5 cut)
        h1_2 = relu(4 x16 + x17 + x19 - 0.5)   A: 2.5    B: 1
        h1_3 = relu(5 x22)                     A: 1      B: 0
        h1_4 = relu(x2 - 2 x18 + 0.25)         A: 0.25   B: 0     (B: -0.25 cut)
        h2_0 = relu(h1_0 + h1_2 - 1)           A: 2.5    B: 0
        h2_1 = relu(-h1_2 + 0.5)               A: 0      B: 0     (A: -2 cut)
        h2_2 = relu(2 h1_3 + 4 h1_4)           A: 3      B: 0
        h2_3 = relu(h1_1 + 3)                  A: 3      B: 3.5
        z = h2_0 + 7 h2_1 - 0.5 h2_2 + 0.25 h2_3 - 1
                                               A: 0.75   B: -0.125

    A dropped ReLU, a missing bias, a transposed weight matrix or argument
    bits read in the wrong order each change z."""
    n_sym = 2
    P = {k: np.zeros(s) for k, s in M.param_shapes(n_sym).items()}
    P["E"][0, 0], P["E"][0, 1], P["E"][1, 2] = 0.5, -1.0, 1.5
    W1, b1, W2, b2 = P["W1"], P["b1"], P["W2"], P["b2"]
    W1[0, 0] = 2
    W1[1, 1], b1[1] = 1, 0.5
    W1[2, 16], W1[2, 17], W1[2, 19], b1[2] = 4, 1, 1, -0.5
    W1[3, 22] = 5
    W1[4, 2], W1[4, 18], b1[4] = 1, -2, 0.25
    W2[0, 0], W2[0, 2], b2[0] = 1, 1, -1
    W2[1, 2], b2[1] = -1, 0.5
    W2[2, 3], W2[2, 4] = 2, 4
    W2[3, 1], b2[3] = 1, 3
    P["w3"][:4] = [1, 7, -0.5, 0.25]
    P["b3"][0] = -1
    # every weight is exactly representable in bfloat16
    for v in P.values():
        assert np.array_equal(M.bf16_round(v), v)
    loss, p, _ = M.forward_backward(P, [0, 1], [2, 1], [0b00101, 0b11110], [3, 0], [1, 0])
    zA, zB = 0.75, -0.125
    sig = lambda z: 1.0 / (1.0 + math.exp(-z))
    assert p[0] == pytest.approx(sig(zA), rel=1e-12)
    assert p[1] == pytest.approx(sig(zB), rel=1e-12)
    # binary cross-entropy: A (label 1) -log p_A, B (label 0) -log(1 - p_B)
    want = 0.5 * (-math.log(sig(zA)) - math.log(1.0 - sig(zB)))
    assert loss == pytest.approx(want, rel=1e-12)
