"""Helpers for the GPU parity tests: run the HIP path through the C-ABI
binding, run the oracle on the same inputs, compare."""

from __future__ import annotations

import sys

import numpy as np

from oracle import oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(trs, terms, pool_slots, maxarity=0, predictor=None, **opts):
    from paper_2009_07174_amd import trs as T
    ctx = T.Context(pool_slots, maxarity)
    try:
        ctx.load_trs(trs)
        if predictor is not None:
            ctx.set_predictor(predictor)
        ctx.load_term_list(list(terms))
        st = ctx.normalize(**opts)
        nfs = [ctx.read_nf(i) for i in range(len(terms))]
        counts = ctx.rule_counts()
    finally:
        ctx.close()
    return nfs, counts, st


def run_oracle(trs, terms):
    res = O.normalize_many(trs, terms)
    counts = np.sum([r.counts for r in res], axis=0) if res else np.zeros(len(trs.rules), np.int64)
    return [r.nf for r in res], counts


def assert_parity(trs, terms, pool_slots, maxarity=0, label="", predictor=None, **opts):
    say(f"[parity] {label}: {len(terms)} terms, {sum(len(t) for t in terms)} nodes, opts={opts}")
    nfs, counts, st = run_gpu(trs, terms, pool_slots, maxarity, predictor=predictor, **opts)
    say(f"[parity] {label}: gpu rounds={st['rounds']} apps={st['rule_apps']} ms={st['device_ms']:.2f}")
    onfs, ocounts = run_oracle(trs, terms)
    for i, (a, b) in enumerate(zip(nfs, onfs)):
        if not np.array_equal(a, b):
            raise AssertionError(f"{label}: term {i}: normal forms differ (gpu len {len(a)}, "
                                 f"oracle len {len(b)})")
    np.testing.assert_array_equal(counts, ocounts, err_msg=f"{label}: per-rule counts")
    assert st["rule_apps"] == int(ocounts.sum())
    return st
