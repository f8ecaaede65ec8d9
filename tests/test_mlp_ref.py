"""Pins for the CPU reference of the frontier predictor: central finite
differences of its own loss, closed-form special cases, bfloat16 rounding."""

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
