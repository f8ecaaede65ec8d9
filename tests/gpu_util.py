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


def run_oracle_parallel(trs, terms, threads: int = 16):
    """The oracle on every term of a batch (independent terms), a thread per
    host core up to ``threads``, each with an oracle of its own; the C
    library releases the interpreter lock while it normalises.  Returns
    (normal forms in term order, per-rule counts summed over the batch)."""
    import os
    import threading
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    nt = max(1, min(threads, cores, len(terms)))
    nfs = [None] * len(terms)
    counts = [None] * nt
    nxt = {"i": 0}
    lock = threading.Lock()

    def worker(k):
        o = O.Oracle.from_trs(trs)
        c = np.zeros(len(trs.rules), np.int64)
        try:
            while True:
                with lock:
                    i = nxt["i"]
                    nxt["i"] = i + 1
                if i >= len(terms):
                    break
                r = o.run(terms[i])
                nfs[i] = r.nf
                c += r.counts
        finally:
            o.close()
            counts[k] = c

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(nt)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    return nfs, np.sum(counts, axis=0)


def compare_nfs(label, gpu_nfs, oracle_nfs):
    """Element-wise comparison of the canonical serialisations."""
    assert len(gpu_nfs) == len(oracle_nfs), label
    bad = [i for i, (a, b) in enumerate(zip(gpu_nfs, oracle_nfs)) if not np.array_equal(a, b)]
    if bad:
        i = bad[0]
        raise AssertionError(f"{label}: {len(bad)} of {len(gpu_nfs)} normal forms differ; first "
                             f"term {i} (gpu length {len(gpu_nfs[i])}, oracle length "
                             f"{len(oracle_nfs[i])})")
