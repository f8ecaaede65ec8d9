"""Closed forms that pin the oracle (and, through it, the GPU path).

Everything here is plain integer arithmetic on the *input* terms, written from
what the rewrite systems compute; none of it rewrites terms.  Each helper
returns the expected normal form and the expected number of applications of
each rule, keyed by the rule's left-hand side as printed by
``trs_workloads.term_to_str``.
"""

from __future__ import annotations

from collections import Counter

import numpy as np


def fib(n: int) -> int:
    a, b = 0, 1
    for _ in range(n):
        a, b = b, a + b
    return a


# ---------------------------------------------------------------- g / Fibonacci

def g_counts(n: int) -> Counter:
    """Rule applications for g(S^n(0)) under g(0)->S(0), g(S(0))->S(0),
    g(S(S(x)))->plus(g(S(x)),g(x)) and Peano plus.

    The call tree of g has Fib(n-1) leaves g(0), Fib(n) leaves g(S(0)) and
    Fib(n+1)-1 inner calls; each inner call g(k) ends in plus(g(k-1), g(k-2))
    whose left operand has value Fib(k), costing Fib(k) peeling steps and one
    base step.
    """
    c = Counter()
    # number of calls g(k) made while evaluating g(n)
    calls = [0] * (n + 1)
    calls[n] = 1
    for k in range(n, 1, -1):
        calls[k - 1] += calls[k]
        calls[k - 2] += calls[k]
    c["g(0)"] = calls[0]
    if n >= 1:
        c["g(S(0))"] = calls[1]
    c["g(S(S(X)))"] = sum(calls[2:])
    c["plus(0, Y)"] = sum(calls[2:])
    c["plus(S(X), Y)"] = sum(calls[k] * fib(k) for k in range(2, n + 1))
    return c


# ---------------------------------------------------------------- Peano trees

def peano_eval(trs, code) -> tuple[int, Counter]:
    """Value of a ground plus/times/S/0 term and the rule applications of
    innermost normalisation: plus(a, b) takes a peeling steps and one base
    step; times(a, b) takes a steps of times(S(x), y), one of times(0, y) and
    a additions plus(b, .) of b + 1 steps each."""
    S, Z = trs.sym_id["S"], trs.sym_id["0"]
    P, T = trs.sym_id["plus"], trs.sym_id["times"]
    c = Counter()
    vals: list[int] = []
    # evaluate the prefix code right to left: operands are on the stack
    for x in reversed([int(v) for v in code]):
        if x == Z:
            vals.append(0)
        elif x == S:
            vals.append(vals.pop() + 1)
        elif x == P:
            a = vals.pop()
            b = vals.pop()
            c["plus(S(X), Y)"] += a
            c["plus(0, Y)"] += 1
            vals.append(a + b)
        elif x == T:
            a = vals.pop()
            b = vals.pop()
            c["times(S(X), Y)"] += a
            c["times(0, Y)"] += 1
            c["plus(S(X), Y)"] += a * b
            c["plus(0, Y)"] += a
            vals.append(a * b)
        else:
            raise ValueError("not a Peano term")
    assert len(vals) == 1
    return vals[0], c


def numeral_code(trs, v: int) -> np.ndarray:
    out = np.full(v + 1, trs.sym_id["S"], dtype=np.int32)
    out[-1] = trs.sym_id["0"]
    return out


# ---------------------------------------------------------------- merge sort

def list_values(trs, code) -> list[int]:
    """Values of a ``cons``/``nil`` list of numerals given as prefix code
    (optionally wrapped in ``sort``)."""
    S, Z = trs.sym_id["S"], trs.sym_id["0"]
    cons, nil = trs.sym_id["cons"], trs.sym_id["nil"]
    out, v = [], 0
    code = [int(x) for x in code]
    i = 1 if code and code[0] == trs.sym_id.get("sort", -99) else 0
    while i < len(code):
        x = code[i]
        if x == cons:
            v = 0
        elif x == S:
            v += 1
        elif x == Z:
            out.append(v)
        elif x == nil:
            pass
        else:
            raise ValueError("not a list of numerals")
        i += 1
    return out


def list_code(trs, values) -> np.ndarray:
    S, Z = trs.sym_id["S"], trs.sym_id["0"]
    cons, nil = trs.sym_id["cons"], trs.sym_id["nil"]
    out = []
    for v in values:
        out.append(cons)
        out.extend([S] * int(v))
        out.append(Z)
    out.append(nil)
    return np.asarray(out, dtype=np.int32)


def msort_sim(values) -> tuple[list[int], Counter]:
    """The merge sort the system encodes, run directly on Python lists while
    counting which rule each step of the system would use.

    sort(L) -> sort2(gt(len(L), S(0)), L): len walks the list (one step per
    cell plus one for nil); gt(len, S(0)) takes one gt(S,S) step when the
    length is at least one, then gt(S(x),0) (length >= 2) or gt(0,0)
    (length 1); the empty list takes gt(0,S(y)).  sort2(true, L) splits L into
    the elements at even and odd positions (each even/odd walk takes one step
    per cell and one for nil, alternating between the two rules) and merges
    the sorted halves; every merge step of two non-empty lists compares the
    heads with lt, which peels min(x, y) times and then takes one base step.
    """
    c = Counter()

    def walk(L, start_even: bool):
        # even(L) / odd(L): cell i uses even if (i even) == start_even
        kind = start_even
        for _ in L:
            c["even(cons(X, L))" if kind else "odd(cons(X, L))"] += 1
            kind = not kind
        c["even(nil)" if kind else "odd(nil)"] += 1

    def merge(L, M):
        out = []
        while True:
            if not L:
                c["merge(nil, M)"] += 1
                return out + M
            if not M:
                c["merge(L, nil)"] += 1
                return out + L
            c["merge(cons(X, L), cons(Y, M))"] += 1
            x, y = L[0], M[0]
            c["lt(S(X), S(Y))"] += min(x, y)
            if x == y:
                c["lt(0, 0)"] += 1
            elif x < y:
                c["lt(0, S(Y))"] += 1
            else:
                c["lt(S(X), 0)"] += 1
            if x < y:
                c["merge2(true, cons(X, L), M)"] += 1
                out.append(x)
                L = L[1:]
            else:
                c["merge2(false, L, cons(Y, M))"] += 1
                out.append(y)
                M = M[1:]

    def sort(L):
        c["sort(L)"] += 1
        c["len(cons(X, L))"] += len(L)
        c["len(nil)"] += 1
        if len(L) == 0:
            c["gt(0, S(Y))"] += 1
        else:
            c["gt(S(X), S(Y))"] += 1
            c["gt(S(X), 0)" if len(L) >= 2 else "gt(0, 0)"] += 1
        if len(L) <= 1:
            c["sort2(false, L)"] += 1
            return list(L)
        c["sort2(true, L)"] += 1
        walk(L, True)
        walk(L, False)
        return merge(sort(L[0::2]), sort(L[1::2]))

    return sort(list(values)), c


# ---------------------------------------------------------------- transformation tree

def ttree_counts(depth: int) -> int:
    """Expand(S^N(0)): 2^N - 1 Expand*(S x) steps, 2^N Expand*(0) steps and
    26 letter steps per leaf: 28 * 2^N - 1 in total."""
    return 28 * (1 << depth) - 1


def counts_by_lhs(trs, counts) -> Counter:
    from trs_workloads import term_to_str
    out = Counter()
    for (lhs, _rhs), k in zip(trs.rules, counts):
        out[term_to_str(lhs)] += int(k)
    return out


def expect_counts(trs, expected: Counter) -> np.ndarray:
    """Expected per-rule vector in the system's rule order (rules that a
    closed form does not mention are expected to fire zero times)."""
    from trs_workloads import term_to_str
    keys = [term_to_str(l) for l, _ in trs.rules]
    unknown = set(expected) - set(keys)
    assert not unknown, unknown
    return np.asarray([expected.get(k, 0) for k in keys], dtype=np.int64)
