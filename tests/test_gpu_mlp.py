"""GPU tests of the frontier predictor's kernels against the CPU reference
(oracle/mlp_ref.py, float64): loss, gradients and probabilities of the
forward/backward kernel, the compiled decision table, and training.

Tolerance: the device accumulates every sum in float32 over at most 64 terms
per tile (plus float atomics across tiles); with operands of order 1 the
relative error of a sum of n terms is below n * 2^-24 times the sum of
magnitudes, so 1e-3 relative (plus 1e-5 of the largest gradient, for
entries that cancel to near zero) bounds it with a wide margin.  The
network's weights are bfloat16 on both sides (the reference takes the same
bit patterns)."""

import numpy as np
import pytest

from oracle import mlp_ref as M
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _T():
    from paper_2009_07174_amd import trs as T
    return T


def ref_params(n_sym, seed, bias_scale=0.3):
    p = M.init_params(n_sym, seed)
    rng = np.random.default_rng(seed + 100)
    # biases off zero so that the ReLU kinks are not hit exactly
    p["b1"] = M.bf16_round(rng.normal(0, bias_scale, p["b1"].shape))
    p["b2"] = M.bf16_round(rng.normal(0, bias_scale, p["b2"].shape))
    p["b3"] = M.bf16_round(rng.normal(0, bias_scale, p["b3"].shape))
    return p


def to_bits(params):
    """float64 values (exact bfloat16) -> uint16 bit patterns, C-ABI order."""
    flat = M.flatten(params).astype(np.float32)
    u = flat.view(np.uint32)
    assert np.all(u & 0xFFFF == 0), "values must be exact bfloat16"
    return (u >> 16).astype(np.uint16)


def records(rng, n, n_sym, arity_of):
    sym = rng.integers(0, n_sym, n)
    ar = np.asarray(arity_of)[sym]
    bits = rng.integers(0, 32, n) | (31 << ar) & 31   # positions >= arity set
    bucket = rng.integers(0, 16, n)
    label = rng.integers(0, 2, n)
    return (sym, ar, bits, bucket, label), M.encode_records(sym, ar, bits, bucket, label)


@pytest.mark.parametrize("n,n_sym,seed", [(1, 3, 0), (64, 5, 1), (300, 7, 2), (4097, 15, 3)])
def test_gradients_match_reference(n, n_sym, seed):
    T = _T()
    rng = np.random.default_rng(seed)
    arity = rng.integers(0, 4, n_sym)
    f, rec = records(rng, n, n_sym, arity)
    params = ref_params(n_sym, seed)
    loss, p, g = M.forward_backward(params, *f)
    gl, gg, gp = T.trs_mlp_eval(n_sym, to_bits(params), rec, grads=True, probs=True)
    say(f"[mlp] n={n} loss ref {loss:.6f} gpu {gl:.6f}")
    assert gl == pytest.approx(loss, rel=1e-4, abs=1e-6)
    np.testing.assert_allclose(gp, p, rtol=1e-4, atol=1e-6)
    gref = M.flatten(g)
    np.testing.assert_allclose(gg, gref, rtol=1e-3, atol=1e-5 * np.abs(gref).max())


def test_gradient_catches_a_planted_mistake():
    # the comparison above would see a sign error in one gradient block of
    # the reference: flip d/dW2 in a copy and check that it no longer matches
    T = _T()
    rng = np.random.default_rng(9)
    n_sym = 4
    arity = [0, 1, 2, 3]
    f, rec = records(rng, 256, n_sym, arity)
    params = ref_params(n_sym, 9)
    _, _, g = M.forward_backward(params, *f)
    g["W2"] = -g["W2"]
    _, gg, _ = T.trs_mlp_eval(n_sym, to_bits(params), rec)
    with pytest.raises(AssertionError):
        gref = M.flatten(g)
        np.testing.assert_allclose(gg, gref, rtol=1e-3, atol=1e-5 * np.abs(gref).max())


def test_decision_table_matches_reference():
    T = _T()
    n_sym = 9
    arity = np.array([0, 1, 2, 3, 0, 1, 2, 3, 5])
    params = ref_params(n_sym, 4, bias_scale=1.0)
    pref = M.decision_table(params, n_sym, arity, 0.1)
    th = float(np.median(pref))      # a threshold that splits the inputs
    probs, words = T.trs_mlp_table(arity, to_bits(params), th)
    say(f"[mlp] table: p in [{pref.min():.4f}, {pref.max():.4f}], threshold {th:.4f}")
    np.testing.assert_allclose(probs, pref, rtol=1e-4, atol=1e-6)
    idx = np.arange(n_sym * 512)
    keep = ((words[idx >> 5].astype(np.int64) >> (idx & 31)) & 1).astype(bool)
    want = pref.ravel() >= th
    clear = np.abs(pref.ravel() - th) > 1e-4   # decisions away from the threshold
    assert np.array_equal(keep[clear], want[clear])
    assert 0 < keep.sum() < len(keep)


def test_training_learns_a_simple_rule():
    # label = "all argument bits set" (readiness); the trained network must
    # separate it, and its loss as computed by the reference must agree with
    # the device's own evaluation
    T = _T()
    from paper_2009_07174_amd import predictor as PR
    rng = np.random.default_rng(5)
    n_sym, n = 6, 200_000
    arity = rng.integers(1, 4, n_sym)
    sym = rng.integers(0, n_sym, n)
    ar = arity[sym]
    bits = rng.integers(0, 32, n) | (31 << ar) & 31
    bucket = rng.integers(0, 16, n)
    label = (bits == 31).astype(np.int64)
    rec = M.encode_records(sym, ar, bits, bucket, label)
    w0 = PR.init_params(n_sym, 0)
    l0, _, _ = T.trs_mlp_eval(n_sym, w0, rec, grads=False)
    params, res = T.trs_mlp_train(n_sym, rec, w0, epochs=3, batch=2048, lr=3e-3, val_frac=0.1)
    say(f"[mlp] training: start loss {l0:.4f}, {res}")
    assert res["val_loss"][-1] < 0.05 < l0
    l1, _, pr = T.trs_mlp_eval(n_sym, params, rec[:5000], grads=False, probs=True)
    pd = {k: v for k, v in M.unflatten(
        (params.astype(np.uint32) << 16).view(np.float32).astype(np.float64), n_sym).items()}
    lref, pref, _ = M.forward_backward(pd, sym[:5000], ar[:5000], bits[:5000], bucket[:5000],
                                       label[:5000])
    assert l1 == pytest.approx(lref, rel=1e-3, abs=1e-5)
    np.testing.assert_allclose(pr, pref, rtol=1e-3, atol=1e-5)
    acc = np.mean((pr >= 0.5) == label[:5000].astype(bool))
    assert acc > 0.99


def test_mlp_argument_errors():
    T = _T()
    with pytest.raises(T.TRSError):
        T.trs_mlp_eval(3, np.zeros(T.trs_mlp_param_count(3), np.uint16),
                       np.array([7], np.uint64))  # symbol 7 >= n_sym
    assert T.trs_mlp_param_count(0) == -1
    assert T.trs_mlp_param_count(257) == -1
