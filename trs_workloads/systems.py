"""The rewrite systems used as workloads, in the text form of ``trs_text``.

* ``PEANO``  - Peano addition and multiplication (the paper's Plus examples,
  Section 3, extended with multiplication).
* ``FIB``    - the doubly recursive ``g`` with Peano addition; ``g(S^n(0))``
  normalises to ``S^Fib(n+1)(0)``.
* ``MSORT``  - merge sort over cons/nil lists of Peano numerals, the system of
  Appendix A (merge-sort listing) with the tree wrapper removed and the
  five-argument ``Merge2`` re-expressed with three arguments: the list cells
  ``cons(X, L)`` and ``cons(Y, M)`` are passed whole instead of as their four
  components, so the highest arity is 3.  The right-hand sides are the same
  lists the paper's rules build.
* ``BATCH``  - the union of the three above (one shared signature), used when
  terms of all three kinds are normalised together.
* ``TTREE``  - the transformation-tree system of Appendix A: ``Expand`` and
  ``Expand2`` build a complete binary tree whose leaves each take the chain
  a -> b -> ... -> z -> End (26 steps; the listing writes the letters in
  capitals).
* ``MSORT5`` - the merge-sort system of Appendix A as printed, with the
  five-argument ``Merge2`` and the ``Leaf``/``Node`` tree wrapper.
* Small systems from Section 2 used by the tests: ``STRATEGY`` (the
  ``f(f(x)) -> a`` example) and ``LOOP`` (the non-terminating ``f(a) ->
  f(f(a))``).
"""

from .trs_text import parse_trs

PEANO_RULES = """
eqn plus(0, Y) = Y
eqn plus(S(X), Y) = S(plus(X, Y))
eqn times(0, Y) = 0
eqn times(S(X), Y) = plus(Y, times(X, Y))
"""

G_RULES = """
eqn g(0) = S(0)
eqn g(S(0)) = S(0)
eqn g(S(S(X))) = plus(g(S(X)), g(X))
"""

PLUS_RULES = """
eqn plus(0, Y) = Y
eqn plus(S(X), Y) = S(plus(X, Y))
"""

MSORT_RULES = """
eqn len(nil) = 0
eqn len(cons(X, L)) = S(len(L))
eqn merge(nil, M) = M
eqn merge(L, nil) = L
eqn merge(cons(X, L), cons(Y, M)) = merge2(lt(X, Y), cons(X, L), cons(Y, M))
eqn merge2(true, cons(X, L), M) = cons(X, merge(L, M))
eqn merge2(false, L, cons(Y, M)) = cons(Y, merge(L, M))
eqn sort(L) = sort2(gt(len(L), S(0)), L)
eqn sort2(false, L) = L
eqn sort2(true, L) = merge(sort(even(L)), sort(odd(L)))
eqn even(nil) = nil
eqn even(cons(X, L)) = cons(X, odd(L))
eqn odd(nil) = nil
eqn odd(cons(X, L)) = even(L)
eqn gt(0, 0) = false
eqn gt(0, S(Y)) = false
eqn gt(S(X), 0) = true
eqn gt(S(X), S(Y)) = gt(X, Y)
eqn lt(0, 0) = false
eqn lt(0, S(Y)) = true
eqn lt(S(X), 0) = false
eqn lt(S(X), S(Y)) = lt(X, Y)
"""

PEANO = "sym 0/0 S/1 plus/2 times/2\nvar X Y\n" + PEANO_RULES

FIB = "sym 0/0 S/1 plus/2 g/1\nvar X Y\n" + G_RULES + PLUS_RULES

MSORT = ("sym 0/0 S/1 true/0 false/0 nil/0 cons/2 lt/2 gt/2 len/1 even/1 odd/1 "
         "merge/2 merge2/3 sort/1 sort2/2\nvar X Y L M\n" + MSORT_RULES)

BATCH = ("sym 0/0 S/1 plus/2 times/2 g/1 true/0 false/0 nil/0 cons/2 lt/2 gt/2 "
         "len/1 even/1 odd/1 merge/2 merge2/3 sort/1 sort2/2\nvar X Y L M\n"
         + PEANO_RULES + G_RULES + MSORT_RULES)

# the listing names the letters A..Z; lower case avoids the clash with the
# successor S and the variable X
_LETTERS = [chr(c) for c in range(ord("a"), ord("z") + 1)]

TTREE = ("sym 0/0 S/1 " + " ".join(f"{c}/0" for c in _LETTERS)
         + " End/0 Node/2 Expand/1 Expand2/1\nvar X\n"
         + "eqn Expand(0) = a\n"
         + "eqn Expand(S(X)) = Node(Expand(X), Expand2(X))\n"
         + "eqn Expand2(0) = a\n"
         + "eqn Expand2(S(X)) = Node(Expand(X), Expand2(X))\n"
         + "".join(f"eqn {a} = {b}\n" for a, b in zip(_LETTERS, _LETTERS[1:] + ["End"])))

MSORT5 = """
sym Zero/0 S/1 Len/1 True/0 False/0 Lt/2 Gt/2 Nil/0 Cons/2 Merge/2 Merge2/5
sym Even/1 Odd/1 Sort/1 Sort2/2 Leaf/1 Node/2
var X Y B L M
eqn Len(Nil) = Zero
eqn Len(Cons(X, L)) = S(Len(L))
eqn Merge(Nil, M) = M
eqn Merge(L, Nil) = L
eqn Merge(Cons(X, L), Cons(Y, M)) = Merge2(Lt(X, Y), X, L, Y, M)
eqn Merge2(True, X, L, Y, M) = Cons(X, Merge(L, Cons(Y, M)))
eqn Merge2(False, X, L, Y, M) = Cons(Y, Merge(Cons(X, L), M))
eqn Sort(L) = Sort2(Gt(Len(L), S(Zero)), L)
eqn Sort2(False, L) = L
eqn Sort2(True, L) = Merge(Sort(Even(L)), Sort(Odd(L)))
eqn Even(Nil) = Nil
eqn Even(Cons(X, L)) = Cons(X, Odd(L))
eqn Odd(Nil) = Nil
eqn Odd(Cons(X, L)) = Even(L)
eqn Gt(Zero, Zero) = False
eqn Gt(Zero, S(Y)) = False
eqn Gt(S(X), Zero) = True
eqn Gt(S(X), S(Y)) = Gt(X, Y)
eqn Lt(Zero, Zero) = False
eqn Lt(Zero, S(Y)) = True
eqn Lt(S(X), Zero) = False
eqn Lt(S(X), S(Y)) = Lt(X, Y)
"""

STRATEGY = """
sym f/1 a/0
var X
eqn f(f(X)) = a
"""

LOOP = """
sym f/1 a/0
eqn f(a) = f(f(a))
"""


def peano():
    return parse_trs(PEANO)


def fib():
    return parse_trs(FIB)


def msort():
    return parse_trs(MSORT)


def batch():
    return parse_trs(BATCH)


def ttree():
    return parse_trs(TTREE)


def msort5():
    return parse_trs(MSORT5)
