"""Parity at the benchmark's full sizes: every term's normal form, element by
element, and the per-rule counts, against the oracle.

* the 4096-term batch in its 2^27-slot pool, in every mode (plain full
  sweep, parent-notification frontier, learned frontier with the packaged
  predictor), at the launch shape the benchmark's autotuner picks;
* g(S^30(0)) in its 2^24-slot pool, also pinned by the closed forms
  (Fib(31) S symbols; the call-tree rule counts);
* the batch plus g(S^32(0)) (4097 terms).

The oracle runs on a thread per host core over the batch's independent
terms.  The batch's oracle results are computed once per session.
"""

import numpy as np
import pytest

from trs_workloads import generators as G
from tests import closed_forms as CF
from tests.gpu_util import compare_nfs, run_oracle_parallel, say

pytestmark = pytest.mark.gpu

_ORACLE = {}


def oracle_of(w):
    if w.name not in _ORACLE:
        say(f"[fullsize] oracle on {w.name}: {w.n_terms} terms")
        _ORACLE[w.name] = run_oracle_parallel(w.trs, w.terms)
    return _ORACLE[w.name]


def gpu_run(w, predictor=None, **opts):
    from paper_2009_07174_amd import trs as T
    ctx = T.Context(w.pool_slots, w.maxarity)
    try:
        ctx.load_trs(w.trs)
        if predictor is not None:
            ctx.set_predictor(predictor)
        off, code = w.packed()
        ctx.load_terms(off, code)
        st = ctx.normalize(**opts)
        say(f"[fullsize] {w.name} {opts}: {st['rounds']} rounds, {st['rule_apps']} rule "
            f"applications, {st['device_ms']:.1f} ms")
        nfs = [ctx.read_nf(i) for i in range(w.n_terms)]
        counts = ctx.rule_counts()
    finally:
        ctx.close()
    return nfs, counts, st


def check(w, nfs, counts, st, label):
    onfs, ocounts = oracle_of(w)
    compare_nfs(label, nfs, onfs)
    np.testing.assert_array_equal(counts, ocounts, err_msg=f"{label}: per-rule counts")
    assert st["rule_apps"] == int(ocounts.sum())


# the launch shape the benchmark's autotuner chose for each mode on this batch
SHAPES = {"plain": dict(mode=0, block=128, nodes_per_thread=8),
          "frontier": dict(mode=1, block=128, nodes_per_thread=8),
          "learned": dict(mode=2, block=128, nodes_per_thread=8)}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["frontier", "plain", "learned"])
def test_batch_4096_full_size(mode):
    w = G.cfg3()
    pred = None
    if mode == "learned":
        from paper_2009_07174_amd import predictor as PR
        pred = PR.load(PR.DEFAULT_WEIGHTS, w.trs.symbols)
    nfs, counts, st = gpu_run(w, predictor=pred, **SHAPES[mode])
    check(w, nfs, counts, st, f"{w.name} {mode}")


@pytest.mark.timeout(900)
def test_g30_full_size():
    w = G.cfg1(30)
    nfs, counts, st = gpu_run(w, mode=1)
    np.testing.assert_array_equal(nfs[0], CF.numeral_code(w.trs, CF.fib(31)))
    assert st["rule_apps"] == sum(CF.g_counts(30).values()) == 21_601_675
    np.testing.assert_array_equal(counts, CF.expect_counts(w.trs, CF.g_counts(30)))
    check(w, nfs, counts, st, w.name)


@pytest.mark.timeout(1200)
def test_batch_with_g32_full_size():
    w = G.cfg4()
    nfs, counts, st = gpu_run(w, mode=1, block=128, nodes_per_thread=8)
    np.testing.assert_array_equal(nfs[-1], CF.numeral_code(w.trs, CF.fib(33)))
    check(w, nfs, counts, st, w.name)
