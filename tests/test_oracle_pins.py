"""Pins for the CPU oracle: worked examples of the paper, closed forms,
special cases and rule validation.  Every expected value here comes from the
paper or from plain arithmetic in ``closed_forms.py``, never from the oracle.
"""

import glob
import os

import numpy as np
import pytest

from oracle import oracle as O
from trs_workloads import generators as G
from trs_workloads import parse_trs, systems, term_to_str, decode_prefix
from tests import closed_forms as CF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_fixture(path):
    body, extra = [], {}
    for line in open(path):
        kw = line.split(" ", 1)[0]
        if kw in ("input", "expect", "steps"):
            extra[kw] = line.split(" ", 1)[1].strip()
        else:
            body.append(line)
    return parse_trs("".join(body)), extra


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.trs"))),
                         ids=lambda p: os.path.basename(p))
def test_golden_fixture(path):
    trs, ex = load_fixture(path)
    r = O.normalize(trs, trs.encode(ex["input"]))
    assert term_to_str(decode_prefix(trs, r.nf)) == ex["expect"]
    if "steps" in ex:
        assert r.steps == int(ex["steps"])


def test_strategy_matters_for_nonconfluent_system():
    # Section 2: f(f(x)) -> a on f(f(f(a))) -- innermost must give f(a), not a
    trs = parse_trs(systems.STRATEGY)
    r = O.normalize(trs, trs.encode("f(f(f(a)))"))
    assert term_to_str(decode_prefix(trs, r.nf)) == "f(a)"


def test_nonterminating_system_hits_step_bound():
    # Section 2: f(a) -> f(f(a)) admits an infinite reduction
    trs = parse_trs(systems.LOOP)
    with pytest.raises(O.OracleError) as e:
        O.normalize(trs, trs.encode("f(a)"), max_steps=1000)
    assert e.value.code == O.ORC_E_STEPS


@pytest.mark.parametrize("bad", [
    "sym f/1 a/0\nvar X\neqn X = a\n",                 # Def. 1 (1): lhs is a variable
    "sym f/1 a/0\nvar X Y\neqn f(X) = Y\n",            # Def. 1 (2): Var(r) not in Var(l)
    "sym f/2 a/0\nvar X\neqn f(X, X) = a\n",           # not left-linear
])
def test_rule_validation(bad):
    trs = parse_trs(bad)
    with pytest.raises(O.OracleError) as e:
        O.Oracle.from_trs(trs)
    assert e.value.code == O.ORC_E_RULE


def test_arity_mismatch_rejected():
    trs = systems.peano()
    arity, off, code = trs.encode_rules()
    code = code.copy()
    code[off[1] - 1] = trs.sym_id["plus"]       # rhs of rule 0 loses its operands
    with pytest.raises(O.OracleError):
        O.Oracle(arity, off, code)


def test_nonground_input_rejected():
    trs = systems.peano()
    o = O.Oracle.from_trs(trs)
    with pytest.raises(O.OracleError) as e:
        o.run(np.asarray([trs.sym_id["S"], -1], np.int32))
    assert e.value.code == O.ORC_E_TERM


# ------------------------------------------------------------------ Peano

@pytest.mark.parametrize("seed", range(8))
def test_peano_random_trees(seed):
    trs = systems.peano()
    rng = np.random.default_rng(1000 + seed)
    L = int(rng.integers(2, 200))
    t = G.peano_tree(trs, rng, L)
    v, cnt = CF.peano_eval(trs, t)
    r = O.normalize(trs, t)
    np.testing.assert_array_equal(r.nf, CF.numeral_code(trs, v))
    np.testing.assert_array_equal(r.counts, CF.expect_counts(trs, cnt))


def test_cfg0_closed_form():
    w = G.cfg0()
    v, cnt = CF.peano_eval(w.trs, w.terms[0])
    r = O.normalize(w.trs, w.terms[0])
    assert len(r.nf) == v + 1
    np.testing.assert_array_equal(r.nf, CF.numeral_code(w.trs, v))
    np.testing.assert_array_equal(r.counts, CF.expect_counts(w.trs, cnt))
    assert int(np.sum(w.terms[0] == w.trs.sym_id["times"])) == 102


@pytest.mark.parametrize("a,b", [(0, 0), (0, 3), (3, 0), (2, 5), (7, 4)])
def test_times_special_cases(a, b):
    trs = systems.peano()
    t = trs.encode("times(" + "S(" * a + "0" + ")" * a + ", " + "S(" * b + "0" + ")" * b + ")")
    r = O.normalize(trs, t)
    np.testing.assert_array_equal(r.nf, CF.numeral_code(trs, a * b))
    assert r.steps == a + 1 + a * (b + 1)


# ------------------------------------------------------------------ g / Fibonacci

@pytest.mark.parametrize("n", list(range(0, 16)) + [20, 25])
def test_fib_closed_form(n):
    trs = systems.fib()
    r = O.normalize(trs, G.g_term(trs, n))
    np.testing.assert_array_equal(r.nf, CF.numeral_code(trs, CF.fib(n + 1)))
    np.testing.assert_array_equal(r.counts, CF.expect_counts(trs, CF.g_counts(n)))


def test_fib_tabulated_totals():
    # totals from the recurrences G(n) = 1 + G(n-1) + G(n-2), P(n) = P(n-1) +
    # P(n-2) + Fib(n) + 1 (tabulated for the configurations)
    for n, total in [(20, 126681), (25, 1676377), (30, 21601675), (32, 59706401)]:
        assert sum(CF.g_counts(n).values()) == total


# ------------------------------------------------------------------ merge sort

@pytest.mark.parametrize("seed", range(6))
def test_msort_random_lists(seed):
    trs = systems.msort()
    rng = np.random.default_rng(2000 + seed)
    vals = rng.integers(0, 10, size=int(rng.integers(0, 40))).tolist()
    t = G.sort_term(trs, vals)
    srt, cnt = CF.msort_sim(vals)
    assert srt == sorted(vals)
    r = O.normalize(trs, t)
    np.testing.assert_array_equal(r.nf, CF.list_code(trs, sorted(vals)))
    np.testing.assert_array_equal(r.counts, CF.expect_counts(trs, cnt))


def test_cfg2_closed_form():
    w = G.cfg2()
    vals = CF.list_values(w.trs, w.terms[0])
    assert len(vals) == 4096
    srt, cnt = CF.msort_sim(vals)
    r = O.normalize(w.trs, w.terms[0])
    np.testing.assert_array_equal(r.nf, CF.list_code(w.trs, sorted(vals)))
    np.testing.assert_array_equal(r.counts, CF.expect_counts(w.trs, cnt))
    # data-independent structural counts for a list of 2^12 elements
    byl = CF.counts_by_lhs(w.trs, r.counts)
    assert byl["sort(L)"] == 8191
    assert byl["len(nil)"] + byl["len(cons(X, L))"] == 61439
    assert sum(byl[k] for k in byl if k.startswith(("even", "odd"))) == 106494
    assert sum(byl[k] for k in byl if k.startswith("gt")) == 16382


# ------------------------------------------------------------------ transformation tree

@pytest.mark.parametrize("depth", [0, 1, 3, 6])
def test_ttree_closed_form(depth):
    w = G.ttree(depth)
    r = O.normalize(w.trs, w.terms[0])
    assert r.steps == CF.ttree_counts(depth)
    node, end = w.trs.sym_id["Node"], w.trs.sym_id["End"]
    # a complete binary tree in prefix order: 2^N - 1 Nodes then leaves in
    # a fixed interleaving; check the multiset and the shape via the parser
    assert int(np.sum(r.nf == node)) == (1 << depth) - 1
    assert int(np.sum(r.nf == end)) == 1 << depth
    tree = decode_prefix(w.trs, r.nf)

    def depth_ok(t, d):
        if t[0] == "End":
            return d == 0
        return t[0] == "Node" and depth_ok(t[1][0], d - 1) and depth_ok(t[1][1], d - 1)
    assert depth_ok(tree, depth)


# ------------------------------------------------------------------ paper's full merge sort

def _list5(vs):
    s = "Nil"
    for v in reversed(vs):
        s = f"Cons({'S(' * int(v)}Zero{')' * int(v)}, {s})"
    return s


def _tree5(lists, leaf="Leaf(Sort({}))"):
    level = [leaf.format(_list5(v)) for v in lists]
    while len(level) > 1:
        level = [f"Node({level[i]}, {level[i + 1]})" for i in range(0, len(level), 2)]
    return level[0]


@pytest.mark.parametrize("depth,length", [(0, 5), (2, 3), (3, 5)])
def test_tmsort_generator_matches_the_written_term(depth, length):
    w = G.tmsort(depth, length)
    vals = np.random.default_rng(G.BASE_SEED + 6).integers(0, 10, size=(1 << depth, length))
    assert np.array_equal(w.terms[0], w.trs.encode(_tree5(vals)))
    assert w.maxarity == 5


def test_tmsort_normal_form_is_the_sorted_leaves():
    # every leaf's list sorted by a host sort: the oracle's normal form of the
    # tree, in the paper's own merge-sort system
    w = G.tmsort(3, 5)
    vals = np.random.default_rng(G.BASE_SEED + 6).integers(0, 10, size=(8, 5))
    r = O.normalize(w.trs, w.terms[0])
    want = w.trs.encode(_tree5([sorted(v) for v in vals], leaf="Leaf({})"))
    assert np.array_equal(r.nf, want)

def test_msort5_tree_of_lists():
    trs = systems.msort5()
    rng = np.random.default_rng(7)
    lists = [rng.integers(0, 6, size=5).tolist() for _ in range(4)]

    def lst(vs):
        s = "Nil"
        for v in reversed(vs):
            s = f"Cons({'S(' * v}Zero{')' * v}, {s})"
        return s
    leaves = [f"Leaf(Sort({lst(v)}))" for v in lists]
    term = f"Node(Node({leaves[0]}, {leaves[1]}), Node({leaves[2]}, {leaves[3]}))"
    want = (f"Node(Node(Leaf({lst(sorted(lists[0]))}), Leaf({lst(sorted(lists[1]))})), "
            f"Node(Leaf({lst(sorted(lists[2]))}), Leaf({lst(sorted(lists[3]))})))")
    r = O.normalize(trs, trs.encode(term))
    assert term_to_str(decode_prefix(trs, r.nf)) == want


def test_fnv_matches_python_definition():
    trs = systems.fib()
    r = O.normalize(trs, G.g_term(trs, 12))
    assert r.fnv == O.fnv1a64(r.nf)
