"""GPU parity: the HIP path (through the C-ABI) against the oracle.

Normal forms must be byte-identical canonical serialisations and the rule
applications, per rule, must be equal (the innermost rewrites are the same
whatever the schedule when no right-hand side duplicates a subterm that is
not yet a normal form, which holds for every system used here).
"""

import glob
import os

import numpy as np
import pytest

from trs_workloads import generators as G
from trs_workloads import parse_trs, systems
from tests import closed_forms as CF
from tests.gpu_util import assert_parity, run_gpu, run_oracle, say
from tests.test_oracle_pins import load_fixture

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.trs"))),
                         ids=lambda p: os.path.basename(p))
def test_golden(path):
    trs, ex = load_fixture(path)
    assert_parity(trs, [trs.encode(ex["input"])], 1 << 12, label=os.path.basename(path))


# option sets: the plain sweep, the parent-notification frontier (with the
# constructor walk and same-round continuation, its defaults), the frontier
# without either, and the frontier with the walk but no continuation
MODES = {"plain": dict(mode=0), "frontier": dict(mode=1),
         "frontier_nowalk": dict(mode=1, nf_walk=-1, nf_walk_wide=-1),
         "frontier_nocont": dict(mode=1, cont_passes=-1)}


@pytest.mark.parametrize("mode", MODES)
def test_peano_small_trees(mode):
    trs = systems.peano()
    rng = np.random.default_rng(11)
    terms = [G.peano_tree(trs, rng, int(rng.integers(1, 300))) for _ in range(24)]
    assert_parity(trs, terms, 1 << 18, label=f"peano small {mode}", **MODES[mode])


@pytest.mark.parametrize("mode", MODES)
def test_cfg0(mode):
    w = G.cfg0()
    st = assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"{w.name} {mode}",
                       **MODES[mode])
    v, cnt = CF.peano_eval(w.trs, w.terms[0])
    assert st["rule_apps"] == sum(cnt.values())


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 12, 16])
def test_fib_small(n, mode):
    trs = systems.fib()
    assert_parity(trs, [G.g_term(trs, n)], 1 << 16, label=f"g({n}) {mode}", **MODES[mode])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [20, 25])
def test_cfg1(n, mode):
    w = G.cfg1(n)
    st = assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"{w.name} {mode}",
                       **MODES[mode])
    assert st["rule_apps"] == sum(CF.g_counts(n).values())


@pytest.mark.parametrize("mode", MODES)
def test_msort_small_lists(mode):
    trs = systems.msort()
    rng = np.random.default_rng(12)
    terms = [G.sort_term(trs, rng.integers(0, 64, size=int(rng.integers(0, 70))))
             for _ in range(16)]
    assert_parity(trs, terms, 1 << 20, label=f"msort small {mode}", **MODES[mode])


@pytest.mark.parametrize("mode", MODES)
def test_cfg2(mode):
    w = G.cfg2()
    assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"{w.name} {mode}",
                  **MODES[mode])


@pytest.mark.parametrize("mode", MODES)
def test_batch_mini(mode):
    w = G.cfg3(n_terms=96, pool_slots=1 << 22, scale="mini")
    assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"{w.name} {mode}",
                  **MODES[mode])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("block,npt", [(64, 1), (128, 2), (256, 4), (512, 8), (1024, 16)])
def test_launch_shapes_agree(block, npt, mode):
    w = G.cfg3(n_terms=48, pool_slots=1 << 21, scale="mini")
    assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity,
                  label=f"mini B{block} npt{npt} {mode}", block=block, nodes_per_thread=npt,
                  **MODES[mode])



@pytest.mark.parametrize("mode", [0, 1])
def test_grid_cap_beyond_residency(mode):
    """A grid cap far above what the chip holds at once, on a batch whose
    sweep spans thousands of tiles of 64 slots: the round launches are kept
    within the resident set, so every workgroup reads the published round
    before any working one ends, and the normal forms agree."""
    w = G.cfg3(n_terms=1024, pool_slots=1 << 22, scale="mini")
    assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"grid cap mode {mode}",
                  mode=mode, block=64, nodes_per_thread=1, max_grid=1 << 16)

@pytest.mark.parametrize("mode", MODES)
def test_ttree(mode):
    w = G.ttree(10, pool_slots=1 << 18)
    st = assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"{w.name} {mode}",
                       **MODES[mode])
    assert st["rule_apps"] == CF.ttree_counts(10)


@pytest.mark.parametrize("mode", MODES)
def test_fast_growing_term_resizes_the_grid(mode):
    """A term that doubles every round (transformation tree of depth 15:
    32768 leaves, each rewritten 26 times) starts on the grid sized for its
    first node.  Rounds whose lists or sweep outgrow the grid are skipped by
    the launches and the host captures a larger grid; the results are the
    oracle's and the closed form's."""
    w = G.ttree(15, pool_slots=1 << 20)
    st = assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"{w.name} {mode} B64",
                       **MODES[mode], block=64, nodes_per_thread=1)
    assert st["rule_apps"] == CF.ttree_counts(15)
    # every level's redexes share one numeral, whose reference count the
    # firings update together (combined per wave): the 16 slots of the
    # numeral S^15(0) die, no other slot does, so a lost or doubled
    # decrement shows here
    assert st["frees"] == 16


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("depth", [8, 12])
def test_tree_merge_sort(mode, depth):
    """The paper's tree merge sort (5-argument Merge2, maxarity 5): a tree of
    depth 8 (12) over 256 (4096) lists of 5 values, the generator the
    benchmark uses at depth 23."""
    w = G.tmsort(depth, 5)
    assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"{w.name} {mode}",
                  **MODES[mode])


@pytest.mark.parametrize("mode", MODES)
def test_msort5_arity5(mode):
    trs = systems.msort5()
    rng = np.random.default_rng(5)

    def lst(vs):
        s = "Nil"
        for v in reversed(vs):
            s = f"Cons({'S(' * int(v)}Zero{')' * int(v)}, {s})"
        return s
    terms = []
    for _ in range(6):
        leaves = [f"Leaf(Sort({lst(rng.integers(0, 9, size=7))}))" for _ in range(4)]
        terms.append(trs.encode(f"Node(Node({leaves[0]}, {leaves[1]}), Node({leaves[2]}, {leaves[3]}))"))
    assert_parity(trs, terms, 1 << 16, label=f"msort5 {mode}", **MODES[mode])


def test_already_normal_and_empty():
    trs = systems.peano()
    nfs, counts, st = run_gpu(trs, [trs.encode("S(S(0))"), trs.encode("0")], 1 << 10)
    assert [list(x) for x in nfs] == [list(trs.encode("S(S(0))")), [0]]
    assert counts.sum() == 0
    nfs, counts, st = run_gpu(trs, [], 1 << 10)
    assert nfs == [] and counts.sum() == 0


def test_pool_exhaustion_reports_error():
    from paper_2009_07174_amd import trs as T
    trs = systems.fib()
    with pytest.raises(T.TRSError) as e:
        run_gpu(trs, [G.g_term(trs, 14)], 256)
    assert e.value.code == T.TRS_E_POOL


@pytest.mark.parametrize("mode", MODES)
def test_round_limit_reports_error(mode):
    """f(a) -> f(f(a)) never ends: one new node per round, so a pool of 2^16
    slots outlasts 200 rounds and the device's round limit must stop the
    run with TRS_E_ROUNDS (and nothing else) after exactly 200 rounds."""
    from paper_2009_07174_amd import trs as T
    trs = parse_trs(systems.LOOP)
    with pytest.raises(T.TRSError) as e:
        run_gpu(trs, [trs.encode("f(a)")], 1 << 16, max_rounds=200, **MODES[mode])
    assert e.value.code == T.TRS_E_ROUNDS
    # a limit above the rounds a terminating run needs changes nothing
    t = systems.fib()
    nfs, _, st = run_gpu(t, [G.g_term(t, 12)], 1 << 16, max_rounds=100_000, **MODES[mode])
    np.testing.assert_array_equal(nfs[0], CF.numeral_code(t, CF.fib(13)))
    assert st["rounds"] < 100_000


@pytest.mark.parametrize("mode", MODES)
def test_persistent_kernel_agrees(mode):
    w = G.cfg3(n_terms=48, pool_slots=1 << 21, scale="mini")
    assert_parity(w.trs, w.terms, w.pool_slots, w.maxarity, label=f"mini persistent {mode}",
                  persistent=1, **MODES[mode])


def test_frontier_with_shared_redexes():
    # a right-hand side with two equal subterms that are not normal forms:
    # the compiled rule shares one node between two parents, so only one
    # parent is notified when it becomes a normal form; the other must be
    # found by a full sweep.  The normal form must not depend on that.
    for rhs in ("p(h(X), h(X))", "p(h(X), k(h(X)))"):
        trs = parse_trs(f"""
sym 0/0 S/1 p/2 d/1 h/1 k/1
var X Y
eqn d(X) = {rhs}
eqn h(S(X)) = S(h(X))
eqn h(0) = 0
eqn k(Y) = Y
eqn p(0, Y) = Y
eqn p(S(X), Y) = S(p(X, Y))
""")
        ks = (0, 1, 3, 6)
        terms = [trs.encode("d(" + "S(" * k + "0" + ")" * k + ")") for k in ks]
        for mode in MODES.values():
            nfs, counts, st = run_gpu(trs, terms, 1 << 14, **mode)
            say(f"[shared] {rhs} mode {mode}: full sweeps {st['full_sweeps']}")
            for k, nf in zip(ks, nfs):
                np.testing.assert_array_equal(nf, CF.numeral_code(trs, 2 * k))


def test_repeat_normalize_same_context():
    from paper_2009_07174_amd import trs as T
    trs = systems.fib()
    ctx = T.Context(1 << 16, 0)
    try:
        ctx.load_trs(trs)
        for n in (9, 13, 9):
            ctx.load_term_list([G.g_term(trs, n)])
            ctx.normalize()
            np.testing.assert_array_equal(ctx.read_nf(0), CF.numeral_code(trs, CF.fib(n + 1)))
    finally:
        ctx.close()


def test_autotune_plain_tunes_the_grid():
    from paper_2009_07174_amd import trs as T
    w = G.cfg3(60, 1 << 20, "mini")
    ctx = T.Context(w.pool_slots, w.maxarity)
    try:
        ctx.load_trs(w.trs)
        ctx.load_term_list(w.terms)
        best, res = ctx.autotune(T.Options(mode=0))
        say(f"[autotune plain] {res}")
        assert res["trials"] == 7
        tab = [(b, npt) for b, npt, _, _ in res["table"]]
        assert tab[:4] == [(64, 16), (128, 16), (256, 16), (512, 16)]
        b0 = min(res["table"][:4], key=lambda t: t[3])[0]
        assert tab[4:] == [(b0, 2), (b0, 4), (b0, 8)]
        assert (best.block, best.nodes_per_thread) == (res["best_block"], res["best_npt"])
        ctx.normalize(best)
        nfs = [ctx.read_nf(i) for i in range(len(w.terms))]
    finally:
        ctx.close()
    onfs, _ = run_oracle(w.trs, w.terms)
    assert all(np.array_equal(a, b) for a, b in zip(nfs, onfs))


def test_autotune_picks_a_shape_and_keeps_results():
    from paper_2009_07174_amd import trs as T
    w = G.cfg3(120, 1 << 21, "mini")
    ctx = T.Context(w.pool_slots, w.maxarity)
    try:
        ctx.load_trs(w.trs)
        ctx.load_term_list(w.terms)
        best, res = ctx.autotune(T.Options(mode=1))
        say(f"[autotune] {res}")
        assert res["trials"] == 9
        assert (best.block, best.nodes_per_thread) == (res["best_block"], res["best_npt"])
        assert res["best_ms"] == min(ms for _, _, _, ms in res["table"])
        best2, res2 = ctx.autotune(T.Options(mode=1))   # cached
        assert res2["trials"] == 0 and best2.block == best.block
        ctx.normalize(best)
        nfs = [ctx.read_nf(i) for i in range(len(w.terms))]
    finally:
        ctx.close()
    onfs, _ = run_oracle(w.trs, w.terms)
    assert all(np.array_equal(a, b) for a, b in zip(nfs, onfs))



@pytest.mark.parametrize("case", ["batch_mini", "batch_mini_16_lists", "cfg2", "fib20"])
def test_plain_scan_kernel_agrees(case, monkeypatch):
    """The plain-mode scan kernel (the default) against the sweep inside the
    round kernel (TRS_NO_SCAN=1): a separate launch classifies the slots of
    each large full round and the round kernel then examines the listed
    slots; results and counts equal the oracle's, and the statistics equal
    those of the in-kernel sweep."""
    if case.startswith("batch_mini"):
        # (a pool of 2^24 slots or more makes the scan use 16 lists)
        pool = 1 << 24 if case.endswith("16_lists") else 1 << 22
        w = G.cfg3(200, pool, "mini")
        trs, terms, pool, A = w.trs, w.terms, w.pool_slots, w.maxarity
    elif case == "cfg2":
        trs = systems.msort()
        vals = np.random.default_rng(G.BASE_SEED + 2).integers(0, 64, size=512)
        terms, pool, A = [G.sort_term(trs, vals)], 1 << 22, 3
    else:
        trs = systems.fib()
        terms, pool, A = [G.g_term(trs, 20)], 1 << 20, 2
    opts = dict(mode=0, block=256, nodes_per_thread=16)
    monkeypatch.setenv("TRS_NO_SCAN", "1")
    base = assert_parity(trs, terms, pool, A, label=f"plain sweep {case}", **opts)
    monkeypatch.delenv("TRS_NO_SCAN")
    scan = assert_parity(trs, terms, pool, A, label=f"plain scan {case}", **opts)
    for k in ("rounds", "node_visits", "active_visits", "ready_visits", "full_sweeps", "memo_blocked"):
        assert scan[k] == base[k], k


@pytest.mark.parametrize("case", ["fib18", "sort512", "batch_mini", "tmsort8"])
@pytest.mark.parametrize("mode", [1, 2])
def test_constructor_walk_and_continuation_cut_rounds(case, mode):
    """Frontier modes' defaults against the plain notification frontier:
    (1) the constructor walk -- a node that becomes a normal form marks the
    constructors above it in the same round; (2) same-round continuation --
    a workgroup examines the ready nodes it created (and roots it rewrote
    into ready ones) in further passes of the round (by default in rounds
    one workgroup runs alone; a fourth run takes both into wide rounds).  Normal forms and rule
    counts equal the oracle's in all three settings; each step needs fewer
    rounds (chains of S and cons cells cost one round instead of one per
    cell, and a chain of plus or lt steps runs inside one round)."""
    from paper_2009_07174_amd import predictor as PR
    if case == "fib18":
        trs = systems.fib()
        terms, pool, A = [G.g_term(trs, 18)], 1 << 18, 2
    elif case == "sort512":
        trs = systems.msort()
        vals = np.random.default_rng(G.BASE_SEED + 2).integers(0, 64, size=512)
        terms, pool, A = [G.sort_term(trs, vals)], 1 << 22, 3
    elif case == "tmsort8":
        w = G.tmsort(8, 5)
        trs, terms, pool, A = w.trs, w.terms, w.pool_slots, w.maxarity
    else:
        w = G.cfg3(96, 1 << 22, "mini")
        trs, terms, pool, A = w.trs, w.terms, w.pool_slots, w.maxarity
    pred = PR.init_params(len(trs.symbols), 0) if mode == 2 else None
    off = assert_parity(trs, terms, pool, A, label=f"{case} mode {mode} no walk", mode=mode,
                        nf_walk=-1, nf_walk_wide=-1, predictor=pred)
    walk = assert_parity(trs, terms, pool, A, label=f"{case} mode {mode} walk", mode=mode,
                         cont_passes=-1, predictor=pred)
    both = assert_parity(trs, terms, pool, A, label=f"{case} mode {mode} walk + continuation",
                         mode=mode, predictor=pred)
    # (the same in wide rounds too: longer walks and further passes there)
    wide = assert_parity(trs, terms, pool, A, label=f"{case} mode {mode} wide settings",
                         mode=mode, predictor=pred, nf_walk_wide=16, cont_passes_wide=4)
    assert wide["nf_walked"] > 0
    say(f"[walk] {case} mode {mode}: rounds {off['rounds']} -> {walk['rounds']} -> "
        f"{both['rounds']}, walked {walk['nf_walked']} / {both['nf_walked']}, ms "
        f"{off['device_ms']:.1f} -> {walk['device_ms']:.1f} -> {both['device_ms']:.1f}")
    assert off["nf_walked"] == 0
    assert walk["nf_walked"] > 0 and both["nf_walked"] > 0
    assert walk["rounds"] < off["rounds"]
    assert both["rounds"] <= walk["rounds"]


@pytest.mark.parametrize("case", ["g16", "batch_mini", "ttree12"])
@pytest.mark.parametrize("mode", [0, 1])
def test_fresh_placement(case, mode):
    """Locality placement (place_fresh): new nodes take fresh slots past the
    extent before recycled ones while the extent is below half the pool.
    Results equal the oracle's; the extent grows beyond the recycling run's
    (slots are not reused while there is room) but stays within the pool."""
    if case == "g16":
        trs = systems.fib()
        terms, pool, A = [G.g_term(trs, 16)], 1 << 20, 2
    elif case == "ttree12":
        w = G.ttree(12, pool_slots=1 << 20)
        trs, terms, pool, A = w.trs, w.terms, w.pool_slots, w.maxarity
    else:
        w = G.cfg3(96, 1 << 22, "mini")
        trs, terms, pool, A = w.trs, w.terms, w.pool_slots, w.maxarity
    base = assert_parity(trs, terms, pool, A, label=f"{case} mode {mode} recycled first", mode=mode)
    fresh = assert_parity(trs, terms, pool, A, label=f"{case} mode {mode} fresh first", mode=mode,
                          place_fresh=50)
    say(f"[placement] {case} mode {mode}: peak {base['peak_slots']} -> {fresh['peak_slots']}, "
        f"ms {base['device_ms']:.1f} -> {fresh['device_ms']:.1f}")
    assert fresh["peak_slots"] >= base["peak_slots"]
    assert fresh["peak_slots"] <= pool
