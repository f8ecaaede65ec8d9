"""GPU tests of trace logging and of learned mode (the frontier chosen by the
predictor).

Learned mode must give exactly the oracle's normal forms and per-rule counts
whatever the predictor says -- keep every candidate, keep none, or a random
or trained network -- because only a full sweep that finds nothing left to
rewrite ends a run.  The trace records of a tiny term are checked against a
hand derivation of the rounds, and the gain test measures what a network
trained on plain-run traces saves over the plain method and over the two
trivial predictors."""

import numpy as np
import pytest

from oracle import mlp_ref as M
from trs_workloads import generators as G
from trs_workloads import systems
from tests.gpu_util import assert_parity, run_gpu, say

pytestmark = pytest.mark.gpu

LEARNED = 2


def _T():
    from paper_2009_07174_amd import trs as T
    return T


def const_predictor(n_sym):
    """All-zero parameters: p = 1/2 for every input."""
    return np.zeros(_T().trs_mlp_param_count(n_sym), np.uint16)


def random_predictor(n_sym, seed):
    from paper_2009_07174_amd import predictor as PR
    return PR.init_params(n_sym, seed)


# ------------------------------------------------------------------ traces

def test_trace_records_of_a_tiny_term():
    """plus(S(0), plus(S(0), 0)) (= 2) in plain mode, every blocked
    node-round logged.  Rounds (a node rewritten or made a normal form in round r is
    seen as such from round r+1; initial nodes changed last in round 0):
      r0: outer plus blocked on arg 1            -> (plus, 2, 0b11101, age 0), label 0
          inner plus(S(0),0) -> S(plus(0,0))
      r1: outer blocked                          -> (plus, .., age 1), label 0
          S blocked on plus(0,0)                 -> (S, 1, 0b11110, age 1), label 1
          plus(0,0) -> 0
      r2: outer blocked                          -> (plus, .., age 2), label 1
          S becomes a normal form
      r3: outer plus(S(0),S(0)) -> S(plus(0,S(0)))
      r4: S blocked                              -> (S, 1, 0b11110, age 1), label 1
          plus(0,S(0)) -> S(0)
      r5: S becomes a normal form."""
    T = _T()
    trs = systems.peano()
    term = trs.encode("plus(S(0), plus(S(0), 0))")
    ctx = T.Context(1 << 10)
    try:
        ctx.load_trs(trs)
        ctx.load_term_list([term])
        st = ctx.normalize(mode=0, trace=65536, label_horizon=1)
        rec = ctx.read_trace()
        nf = ctx.read_nf(0)
    finally:
        ctx.close()
    assert list(nf) == list(trs.encode("S(S(0))"))
    plus, S = trs.sym_id["plus"], trs.sym_id["S"]
    want = sorted([(plus, 2, 0b11101, 0, 0), (plus, 2, 0b11101, 1, 0), (S, 1, 0b11110, 1, 1),
                   (plus, 2, 0b11101, 2, 1), (S, 1, 0b11110, 1, 1)])
    got = sorted(zip(*[list(map(int, f)) for f in M.decode_records(rec)]))
    say(f"[trace] {got}")
    assert got == want
    assert st["trace_records"] == 5


@pytest.mark.parametrize("name", ["g12", "mini_batch"])
def test_trace_keeps_results_and_records_are_valid(name):
    T = _T()
    if name == "g12":
        trs = systems.fib()
        terms, pool = [G.g_term(trs, 12)], 1 << 16
    else:
        w = G.cfg3(60, 1 << 20, "mini")
        trs, terms, pool = w.trs, w.terms, w.pool_slots
    st = assert_parity(trs, terms, pool, label=f"trace {name}", mode=0, trace=65536)
    ctx = T.Context(pool)
    try:
        ctx.load_trs(trs)
        ctx.load_term_list(terms)
        st2 = ctx.normalize(mode=0, trace=20000, trace_cap=1000)
        rec = ctx.read_trace()
    finally:
        ctx.close()
    assert st["trace_records"] > 0
    sym, ar, bits, bucket, label = M.decode_records(rec)
    arity = np.array(trs.arity)
    assert len(rec) == min(1000, st2["trace_records"])
    assert np.all(sym < len(trs.symbols))
    assert np.array_equal(ar, arity[sym])
    assert np.all((bits | ((1 << ar) - 1)) == 31)   # positions >= arity are set
    assert np.all(bits != 31)                        # the node was blocked
    assert np.all(bucket <= 15)
    assert set(np.unique(label)) <= {0, 1}


def test_trace_argument_checks():
    T = _T()
    trs = systems.peano()
    ctx = T.Context(1 << 10)
    try:
        ctx.load_trs(trs)
        ctx.load_term_list([trs.encode("plus(0, 0)")])
        with pytest.raises(T.TRSError):
            ctx.normalize(mode=1, trace=100)      # traces come from plain runs
        with pytest.raises(T.TRSError):
            ctx.normalize(mode=0, trace=70000)
        with pytest.raises(T.TRSError):
            ctx.normalize(mode=LEARNED)           # no predictor installed
    finally:
        ctx.close()


# ------------------------------------------------------------- learned mode

KEEP = {"all": 0.4, "none": 0.6}   # thresholds around the constant p = 1/2


@pytest.mark.parametrize("keep", ["all", "none", "random"])
def test_learned_parity_small(keep):
    cases = []
    trs = systems.peano()
    rng = np.random.default_rng(21)
    cases.append(("peano trees", trs, [G.peano_tree(trs, rng, int(rng.integers(1, 200)))
                                       for _ in range(12)], 1 << 18))
    trs = systems.fib()
    cases.append(("g 0..14", trs, [G.g_term(trs, n) for n in range(15)], 1 << 18))
    trs = systems.msort()
    cases.append(("msort lists", trs, [G.sort_term(trs, rng.integers(0, 64, int(k)))
                                       for k in rng.integers(0, 60, 10)], 1 << 20))
    trs = systems.msort5()

    def lst(vs):
        s = "Nil"
        for v in reversed(vs):
            s = f"Cons({'S(' * int(v)}Zero{')' * int(v)}, {s})"
        return s
    cases.append(("msort5", trs, [trs.encode(f"Node(Leaf(Sort({lst(rng.integers(0, 9, 9))})), "
                                             f"Leaf(Sort({lst(rng.integers(0, 9, 6))})))")
                                  for _ in range(4)], 1 << 18))
    w = G.ttree(10, 1 << 18)
    cases.append(("ttree", w.trs, w.terms, w.pool_slots))
    evals = 0
    for label, trs, terms, pool in cases:
        n_sym = len(trs.symbols)
        if keep == "random":
            pred, th = random_predictor(n_sym, 3), 0.1
        else:
            pred, th = const_predictor(n_sym), KEEP[keep]
        st = assert_parity(trs, terms, pool, label=f"learned {keep} {label}", predictor=pred,
                           mode=LEARNED, threshold=th)
        # (the predictor decides for blocked nodes whose symbol has rules; a
        # system whose only blocked nodes are constructors asks it nothing)
        evals += st["mlp_evals"]
        if keep == "none":
            assert st["mlp_kept"] == 0
        if keep == "all":
            assert st["mlp_kept"] == st["mlp_evals"]
    assert evals > 0


@pytest.mark.parametrize("keep", ["all", "none", "random"])
def test_learned_parity_mini_batch(keep):
    w = G.cfg3(200, 1 << 22, "mini")
    n_sym = len(w.trs.symbols)
    pred = random_predictor(n_sym, 7) if keep == "random" else const_predictor(n_sym)
    th = 0.1 if keep == "random" else KEEP[keep]
    assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"learned {keep} mini batch",
                  predictor=pred, mode=LEARNED, threshold=th)


def test_learned_repeat_and_predictor_swap():
    # the same context normalises again after a new predictor is installed
    T = _T()
    trs = systems.fib()
    term = G.g_term(trs, 13)
    ctx = T.Context(1 << 18)
    try:
        ctx.load_trs(trs)
        ctx.load_term_list([term])
        outs = []
        for k, (pred, th) in enumerate([(const_predictor(4), 0.4), (random_predictor(4, 1), 0.1),
                                        (const_predictor(4), 0.6)]):
            ctx.set_predictor(pred)
            ctx.normalize(mode=LEARNED, threshold=th)
            outs.append(ctx.read_nf(0))
        with pytest.raises(T.TRSError):
            ctx.set_predictor(np.zeros(5, np.uint16))   # wrong parameter count
    finally:
        ctx.close()
    assert all(np.array_equal(o, outs[0]) for o in outs)


# ------------------------------------------------------------------ gain

def test_trained_predictor_gain():
    """Train on plain-run traces (g, sort and a small batch, batch-system
    numbering), then run a held-out batch in plain mode, in learned mode with
    the trained network, in the same frontier without the network (parent
    notification alone: the ablation), and with the two trivial predictors
    (keep every candidate, keep none), all learned runs without periodic
    sweeps.  Results are identical in every run.

    What the network gains: notification already queues every node whose
    last argument becomes a normal form (a node that is not yet a normal
    form has one parent, which the hint reaches), so a blocked node polled
    again before that notification is still blocked.  The network's only
    lever is such polls, and it cannot remove any of the ablation's work.
    The measured ordering is asserted: the ablation visits the fewest nodes,
    the trained network at most as many as keeping every candidate, all of
    them far fewer than the plain sweep."""
    from paper_2009_07174_amd import predictor as PR
    recs = []
    for name, trs, terms, pool, share in PR.training_sets("mini"):
        recs.append(PR.collect(trs, terms, pool, 60_000, log=say))
    rec = np.concatenate(recs)
    n_sym = len(trs.symbols)
    params, res = PR.train(n_sym, rec, epochs=3, log=say)
    assert res["val_loss"][-1] < res["train_loss"][0]
    # held out: a different batch (other seeds) of the same recipe
    w = G.cfg3(300, 1 << 22, "mini")
    terms = w.terms[100:]
    runs = {}
    runs["plain"] = assert_parity(w.trs, terms, w.pool_slots, 3, label="gain plain", mode=0)
    runs["ablation"] = assert_parity(w.trs, terms, w.pool_slots, 3, label="gain no network",
                                     mode=1)
    runs["trained"] = assert_parity(w.trs, terms, w.pool_slots, 3, label="gain trained",
                                    predictor=params, mode=LEARNED, threshold=0.1,
                                    sweep_every=-1)
    runs["keep_all"] = assert_parity(w.trs, terms, w.pool_slots, 3, label="gain keep all",
                                     predictor=const_predictor(n_sym), mode=LEARNED,
                                     threshold=0.4, sweep_every=-1)
    runs["keep_none"] = assert_parity(w.trs, terms, w.pool_slots, 3, label="gain keep none",
                                      predictor=const_predictor(n_sym), mode=LEARNED,
                                      threshold=0.6, sweep_every=-1)
    for k, st in runs.items():
        say(f"[gain] {k}: rounds {st['rounds']} visits {st['node_visits']} full "
            f"{st['full_sweeps']} kept {st['mlp_kept']}/{st['mlp_evals']} ms {st['device_ms']:.1f}")
    ab, tr, ka, kn = runs["ablation"], runs["trained"], runs["keep_all"], runs["keep_none"]
    assert kn["mlp_kept"] == 0 and ka["mlp_kept"] == ka["mlp_evals"]
    assert ab["node_visits"] <= kn["node_visits"] <= tr["node_visits"] <= ka["node_visits"]
    assert tr["node_visits"] * 2 < runs["plain"]["node_visits"]
