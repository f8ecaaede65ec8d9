"""Brute-force pins on tiny terms, independent of the oracle's code.

A plain Python tree rewriter explores *every* rewrite sequence (any redex at
any position, any matching rule) and every innermost sequence.  For the
confluent workload systems the set of reachable normal forms must be a single
term equal to the oracle's, and every maximal innermost sequence must have the
oracle's length (innermost redexes are disjoint, so the order in which a
parallel or sequential rewriter contracts them does not change what is
contracted).  The Section 2 strategy example shows the set is not a singleton
for a non-confluent system, while innermost still gives f(a).
"""

from functools import lru_cache

import numpy as np
import pytest

from oracle import oracle as O
from trs_workloads import generators as G
from trs_workloads import parse_trs, systems, term_to_str, decode_prefix


def to_tuple(t):
    if t[0] == "$var":
        return ("$var", t[1])
    return (t[0], tuple(to_tuple(c) for c in t[1]))


def match(pat, t, env):
    if pat[0] == "$var":
        env[pat[1]] = t
        return True
    if pat[0] != t[0] or len(pat[1]) != len(t[1]):
        return False
    return all(match(p, c, env) for p, c in zip(pat[1], t[1]))


def subst(r, env):
    if r[0] == "$var":
        return env[r[1]]
    return (r[0], tuple(subst(c, env) for c in r[1]))


def redexes(t, rules, path=()):
    """All (position, rule index) pairs where some rule matches."""
    out = []
    for i, (l, _r) in enumerate(rules):
        if match(l, t, {}):
            out.append((path, i))
    for j, c in enumerate(t[1]):
        out.extend(redexes(c, rules, path + (j,)))
    return out


def replace(t, path, new):
    if not path:
        return new
    kids = list(t[1])
    kids[path[0]] = replace(kids[path[0]], path[1:], new)
    return (t[0], tuple(kids))


def at(t, path):
    for j in path:
        t = t[1][j]
    return t


def contract(t, path, rule, rules):
    l, r = rules[rule]
    env = {}
    assert match(l, at(t, path), env)
    return replace(t, path, subst(r, env))


def all_normal_forms(t0, rules, limit=200000):
    seen, nfs, stack = set(), set(), [t0]
    while stack:
        t = stack.pop()
        if t in seen:
            continue
        seen.add(t)
        assert len(seen) < limit, "state space too large for brute force"
        rs = redexes(t, rules)
        if not rs:
            nfs.add(t)
        for p, i in rs:
            stack.append(contract(t, p, i, rules))
    return nfs


def innermost_lengths(t0, rules):
    """Set of lengths of all maximal innermost derivations: at each step pick
    any redex with no redex strictly below it, contracted with the first
    matching rule (the rule priority)."""

    @lru_cache(maxsize=None)
    def lengths(t):
        rs = redexes(t, rules)
        if not rs:
            return frozenset([0])
        firsts = {}
        for p, i in rs:
            if p not in firsts:
                firsts[p] = i
        inner = [p for p in firsts if not any(q != p and q[:len(p)] == p for q in firsts)]
        out = set()
        for p in inner:
            for k in lengths(contract(t, p, firsts[p], rules)):
                out.add(k + 1)
        return frozenset(out)

    return lengths(t0)


def rules_of(trs):
    return [(to_tuple(l), to_tuple(r)) for l, r in trs.rules]


def check(trs, term_text, all_orders=True):
    rules = rules_of(trs)
    t = to_tuple(trs.term(term_text))
    res = O.normalize(trs, trs.encode(term_text))
    if all_orders:
        nfs = all_normal_forms(t, rules)
        assert len(nfs) == 1, f"{len(nfs)} normal forms"
        (nf,) = nfs
        assert to_tuple(decode_prefix(trs, res.nf)) == nf
    lens = innermost_lengths(t, rules)
    assert lens == {res.steps}, (lens, res.steps)


def num(k):
    return "S(" * k + "0" + ")" * k


@pytest.mark.parametrize("term", [
    f"plus({num(2)}, {num(1)})",
    f"times({num(2)}, {num(2)})",
    f"plus(times({num(1)}, {num(2)}), plus({num(2)}, {num(0)}))",
    f"times(plus({num(1)}, {num(1)}), {num(2)})",
])
def test_peano_all_orders(term):
    check(systems.peano(), term)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4])
def test_fib_all_orders(n):
    check(systems.fib(), f"g({num(n)})")


@pytest.mark.parametrize("vals", [[], [1], [2, 0], [1, 1], [2, 0, 1], [0, 2, 1]])
def test_msort_all_orders(vals):
    # every order for lists of up to two elements; for three elements the
    # unrestricted state space is too large, so only innermost orders
    lst = "nil"
    for v in reversed(vals):
        lst = f"cons({num(v)}, {lst})"
    check(systems.msort(), f"sort({lst})", all_orders=len(vals) <= 2)


def test_nonconfluent_example_has_two_normal_forms():
    trs = parse_trs(systems.STRATEGY)
    rules = rules_of(trs)
    nfs = all_normal_forms(to_tuple(trs.term("f(f(f(a)))")), rules)
    assert {term_to_str(_untuple(t)) for t in nfs} == {"a", "f(a)"}
    # innermost still reaches only f(a), in one step
    assert innermost_lengths(to_tuple(trs.term("f(f(f(a)))")), rules) == {1}


def _untuple(t):
    return (t[0], [_untuple(c) for c in t[1]])
