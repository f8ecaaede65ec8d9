"""Invariants of the node pool after a run, read back through
trs_read_pool (Section 3: reference counts, collection of nodes whose count
reaches zero, and reuse of their indices from the free list).

After every normalisation, in every mode:
  * every live slot is a normal form and every argument of a live slot is a
    live slot below the extent n;
  * each live slot's count equals the references to it from the arguments
    of live slots plus the term roots that name it (nothing leaked, nothing
    freed early);
  * every live slot is reachable from a root (collection is complete);
  * the free stacks hold distinct indices in 1..n-1, exactly the slots below
    n that are not live.
The checks are plain host code over the arrays; they share nothing with the
kernels.
"""

import numpy as np
import pytest

from trs_workloads import generators as G
from trs_workloads import systems
from tests.gpu_util import assert_parity, say

pytestmark = pytest.mark.gpu

MODES = {"plain": dict(mode=0), "frontier": dict(mode=1),
         "frontier_nowalk": dict(mode=1, nf_walk=-1, nf_walk_wide=-1),
         "frontier_nocont": dict(mode=1, cont_passes=-1),
         "frontier_wide": dict(mode=1, nf_walk_wide=8, cont_passes_wide=4),
         "frontier_fresh": dict(mode=1, place_fresh=50),
         "plain_fresh": dict(mode=0, place_fresh=50),
         "learned": dict(mode=2)}


def check_pool(pool, arity):
    n, hss, args, state, rc = pool["n"], pool["hss"], pool["args"], pool["state"], pool["rc"]
    roots = pool["roots"]
    assert n >= 1
    live = state != 0
    live[0] = False  # slot 0 is never used
    idx = np.nonzero(live)[0]
    assert np.all((state[idx] & 0x80) != 0), "a live slot is not a normal form"
    assert np.all((hss[idx] >= 0) & (hss[idx] < len(arity))), "bad symbol"
    ar = np.asarray(arity, np.int64)[hss[idx]]
    refs = np.zeros(n, np.int64)
    # argument entries of live slots within their arity
    A = args.shape[1]
    for j in range(A):
        sel = idx[ar > j]
        c = args[sel, j].astype(np.int64)
        assert np.all((c >= 1) & (c < n)), f"argument {j} of a live slot out of range"
        assert np.all(live[c]), f"argument {j} of a live slot is not live"
        np.add.at(refs, c, 1)
    r = roots.astype(np.int64)
    assert np.all((r >= 1) & (r < n)) and np.all(live[r]), "a root is not live"
    np.add.at(refs, r, 1)
    bad = idx[rc[idx] != refs[idx]]
    assert bad.size == 0, (f"{bad.size} live slots with a wrong count; first {bad[0]}: "
                           f"count {rc[bad[0]]}, references {refs[bad[0]]}")
    # reachability from the roots
    seen = np.zeros(n, bool)
    seen[r] = True
    front = np.unique(r)
    while front.size:
        far = np.asarray(arity, np.int64)[hss[front]]
        nxt = [args[front[far > j], j].astype(np.int64) for j in range(A)]
        nxt = np.unique(np.concatenate(nxt)) if nxt else np.zeros(0, np.int64)
        nxt = nxt[~seen[nxt]]
        seen[nxt] = True
        front = nxt
    assert np.array_equal(seen, live), (f"{int((live & ~seen).sum())} live slots unreachable "
                                        "from the roots")
    free = np.concatenate([pool["free0"], pool["free1"]]).astype(np.int64)
    assert np.unique(free).size == free.size, "a free index appears twice"
    assert np.all((free >= 1) & (free < n)), "a free index outside 1..n-1"
    assert np.array_equal(np.sort(free), np.nonzero(~live[1:])[0] + 1), \
        "the free stacks are not exactly the unused slots below n"
    return int(idx.size), int(free.size)


def run_and_check(trs, terms, pool_slots, A, label, **opts):
    from paper_2009_07174_amd import predictor as PR
    from paper_2009_07174_amd import trs as T
    assert_parity(trs, terms, pool_slots, A, label=label, **opts,
                  predictor=PR.init_params(len(trs.symbols), 0) if opts.get("mode") == 2 else None)
    ctx = T.Context(pool_slots, A)
    try:
        ctx.load_trs(trs)
        if opts.get("mode") == 2:
            ctx.set_predictor(PR.init_params(len(trs.symbols), 0))
        ctx.load_term_list(list(terms))
        st = ctx.normalize(**opts)
        pool = ctx.read_pool()
    finally:
        ctx.close()
    nlive, nfree = check_pool(pool, trs.arity)
    say(f"[invariants] {label}: n {pool['n']}, live {nlive}, free {nfree}, "
        f"frees {st['frees']}, peak {st['peak_slots']}")
    assert nfree + nlive == pool["n"] - 1


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", ["cfg0", "g12", "batch_mini", "ttree10", "msort_small"])
def test_pool_invariants(case, mode):
    if case == "cfg0":
        w = G.cfg0()
        trs, terms, pool, A = w.trs, w.terms, w.pool_slots, w.maxarity
    elif case == "g12":
        trs = systems.fib()
        terms, pool, A = [G.g_term(trs, 12)], 1 << 16, 2
    elif case == "batch_mini":
        w = G.cfg3(96, 1 << 22, "mini")
        trs, terms, pool, A = w.trs, w.terms, w.pool_slots, w.maxarity
    elif case == "ttree10":
        w = G.ttree(10, pool_slots=1 << 18)
        trs, terms, pool, A = w.trs, w.terms, w.pool_slots, w.maxarity
    else:
        trs = systems.msort()
        rng = np.random.default_rng(12)
        terms = [G.sort_term(trs, rng.integers(0, 64, size=int(rng.integers(0, 70))))
                 for _ in range(16)]
        pool, A = 1 << 20, 3
    run_and_check(trs, terms, pool, A, f"{case} {mode}", **MODES[mode])
