"""The allocation-free predictor evaluation (trs_mlp_eval_noalloc) against
trs_mlp_eval, through the C-ABI, on two calls in a row -- the second with
fewer records and symbols, so stale contents of the shared static buffer
(the first call's gradient, loss and probabilities) would show -- and both
against the float64 reference.

Tolerance: the two entry points run the same kernel on the same inputs; only
the order of the float32 atomic additions across workgroups may differ, so
the results agree to a few float32 ulps of the accumulated sums (1e-5
relative, plus 1e-6 of the largest gradient for entries that cancel).  The
reference bound is that of the predictor kernel tests (1e-3 relative, plus
1e-5 of the largest gradient)."""

import numpy as np
import pytest

from oracle import mlp_ref as M
from tests.gpu_util import say
from tests.test_gpu_mlp import records, ref_params, to_bits

pytestmark = pytest.mark.gpu


def _T():
    from paper_2009_07174_amd import trs as T
    return T


def test_noalloc_matches_eval_on_two_calls():
    T = _T()
    cases = [(40_000, 200, 21), (700, 6, 22)]   # (records, symbols, seed)
    for n, n_sym, seed in cases:
        rng = np.random.default_rng(seed)
        arity = rng.integers(0, 4, n_sym)
        f, rec = records(rng, n, n_sym, arity)
        params = ref_params(n_sym, seed)
        bits = to_bits(params)
        l0, g0, p0 = T.trs_mlp_eval(n_sym, bits, rec, grads=True, probs=True)
        l1, g1, p1 = T.trs_mlp_eval_noalloc(n_sym, bits, rec, grads=True, probs=True)
        say(f"[noalloc] n={n} n_sym={n_sym}: loss {l0:.7f} / {l1:.7f}")
        assert l1 == pytest.approx(l0, rel=1e-5, abs=1e-7)
        np.testing.assert_allclose(p1, p0, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(g1, g0, rtol=1e-5, atol=1e-6 * np.abs(g0).max())
        loss, p, g = M.forward_backward(params, *f)
        gref = M.flatten(g)
        assert l1 == pytest.approx(loss, rel=1e-4, abs=1e-6)
        np.testing.assert_allclose(p1, p, rtol=1e-4, atol=1e-6)
        np.testing.assert_allclose(g1, gref, rtol=1e-3, atol=1e-5 * np.abs(gref).max())
    # loss only (no gradient, no probabilities) after the two calls above
    l2, g2, p2 = T.trs_mlp_eval_noalloc(n_sym, bits, rec, grads=False, probs=False)
    assert g2 is None and p2 is None
    assert l2 == pytest.approx(l0, rel=1e-5, abs=1e-7)
