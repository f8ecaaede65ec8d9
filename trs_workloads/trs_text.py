"""Text form of a term rewrite system and its integer encoding.

The text form follows the shape of the specification language the paper uses
for its benchmark systems (Section 2, merge-sort example; Appendix A): a list
of function symbols with their arities, a list of variables, and equations
``LHS = RHS`` whose textual order is the rule priority.  Lines::

    sym  name/arity name/arity ...
    var  X Y ...
    eqn  lhs = rhs
    # comment

Terms are written ``f(t1, ..., tk)``; constants may be written ``c`` or
``c()``.

Integer encoding (shared by the C-ABI and the oracle, by specification):

* symbol id = position in the ``sym`` declarations (arity table ``arity[id]``);
* a term is its prefix (pre-order) sequence of symbol ids; arities come from
  the table, so no brackets are stored;
* a rule is the prefix code of its left-hand side immediately followed by the
  prefix code of its right-hand side; a variable is the negative code
  ``-1-k`` where ``k`` numbers the rule's variables in order of first
  occurrence in the left-hand side;
* ``rule_off[i] .. rule_off[i+1]`` delimit rule ``i`` in ``rule_code``.

This module only parses and encodes; validity (Definition 1, left-linearity)
is checked independently by each consumer.
"""

from __future__ import annotations

import re
from dataclasses import dataclass, field

import numpy as np

_TOKEN = re.compile(r"\s*([A-Za-z0-9_']+|\(|\)|,)")


class ParseError(ValueError):
    pass


@dataclass
class TRS:
    symbols: list[str]
    arity: list[int]
    variables: list[str]
    rules: list[tuple[object, object]]          # (lhs, rhs) as nested tuples
    sym_id: dict[str, int] = field(default_factory=dict)

    def __post_init__(self):
        self.sym_id = {s: i for i, s in enumerate(self.symbols)}

    @property
    def maxarity(self) -> int:
        return max(self.arity) if self.arity else 0

    # ----------------------------------------------------------------- encode
    def encode_rules(self):
        """Return ``(arity, rule_off, rule_code)`` as int32 numpy arrays."""
        code: list[int] = []
        off = [0]
        for lhs, rhs in self.rules:
            varnum: dict[str, int] = {}

            def enc(t, in_lhs):
                if t[0] == "$var":
                    name = t[1]
                    if name not in varnum:
                        if not in_lhs:
                            # an RHS-only variable: give it a fresh number so
                            # that the consumer can reject the rule itself
                            varnum[name] = len(varnum)
                        else:
                            varnum[name] = len(varnum)
                    code.append(-1 - varnum[name])
                    return
                code.append(self.sym_id[t[0]])
                for c in t[1]:
                    enc(c, in_lhs)

            enc(lhs, True)
            enc(rhs, False)
            off.append(len(code))
        return (np.asarray(self.arity, dtype=np.int32),
                np.asarray(off, dtype=np.int32),
                np.asarray(code, dtype=np.int32))

    def term(self, text: str):
        """Parse a ground term in this system's syntax."""
        t = _parse_term(text, self)
        return t

    def encode(self, text_or_tree) -> np.ndarray:
        t = self.term(text_or_tree) if isinstance(text_or_tree, str) else text_or_tree
        return encode_term(self, t)

    def rule_index(self, lhs_text: str) -> int:
        """Index of the rule whose left-hand side prints as ``lhs_text``."""
        want = term_to_str(_parse_term(lhs_text, self))
        for i, (l, _r) in enumerate(self.rules):
            if term_to_str(l) == want:
                return i
        raise KeyError(lhs_text)


def _tokens(s: str):
    pos = 0
    out = []
    s = s.strip()
    while pos < len(s):
        m = _TOKEN.match(s, pos)
        if not m:
            raise ParseError(f"bad character at {pos}: {s[pos:pos+10]!r}")
        out.append(m.group(1))
        pos = m.end()
    return out


def _parse_term(text: str, trs: TRS, variables=None):
    variables = set(trs.variables if variables is None else variables)
    toks = _tokens(text)
    # iterative prefix parser (terms may be deep, e.g. long numerals)
    pos = 0

    def parse():
        nonlocal pos
        # explicit stack: frames [name, children, expected]
        root_holder: list = []
        stack = [(None, root_holder, 1)]
        while True:
            if pos >= len(toks):
                raise ParseError("unexpected end of term")
            name = toks[pos]
            pos += 1
            if name in "(),":
                raise ParseError(f"unexpected {name!r}")
            if name in variables:
                node = ("$var", name)
                has_args = pos < len(toks) and toks[pos] == "("
                if has_args:
                    raise ParseError(f"variable {name} applied to arguments")
                stack[-1][1].append(node)
            else:
                if name not in trs.sym_id:
                    raise ParseError(f"unknown symbol {name!r}")
                ar = trs.arity[trs.sym_id[name]]
                if pos < len(toks) and toks[pos] == "(":
                    pos += 1
                    if ar == 0:
                        if pos < len(toks) and toks[pos] == ")":
                            pos += 1
                            stack[-1][1].append((name, []))
                        else:
                            raise ParseError(f"constant {name} given arguments")
                    else:
                        kids: list = []
                        node = (name, kids)
                        stack[-1][1].append(node)
                        stack.append((name, kids, ar))
                        continue
                else:
                    if ar != 0:
                        raise ParseError(f"{name} needs {ar} arguments")
                    stack[-1][1].append((name, []))
            # close finished frames
            while True:
                fname, kids, want = stack[-1]
                if fname is None:
                    return root_holder[0]
                if len(kids) < want:
                    if pos >= len(toks) or toks[pos] != ",":
                        raise ParseError(f"{fname}: expected ',' ")
                    pos += 1
                    break
                if pos >= len(toks) or toks[pos] != ")":
                    raise ParseError(f"{fname}: expected ')'")
                pos += 1
                stack.pop()

    t = parse()
    if pos != len(toks):
        raise ParseError(f"trailing tokens: {toks[pos:pos+5]}")
    return t


def parse_trs(text: str) -> TRS:
    symbols: list[str] = []
    arity: list[int] = []
    variables: list[str] = []
    eqns: list[tuple[str, str]] = []
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        kw, _, rest = line.partition(" ")
        rest = rest.strip()
        if kw == "sym":
            for item in rest.split():
                name, _, a = item.partition("/")
                if not a:
                    raise ParseError(f"symbol {name} without arity")
                if name in symbols:
                    raise ParseError(f"symbol {name} declared twice")
                symbols.append(name)
                arity.append(int(a))
        elif kw == "var":
            variables.extend(rest.split())
        elif kw == "eqn":
            lhs, eq, rhs = rest.partition("=")
            if not eq:
                raise ParseError(f"equation without '=': {line}")
            eqns.append((lhs.strip(), rhs.strip()))
        else:
            raise ParseError(f"unknown keyword {kw!r}")
    trs = TRS(symbols, arity, variables, [])
    for lhs, rhs in eqns:
        trs.rules.append((_parse_term(lhs, trs), _parse_term(rhs, trs)))
    return trs


def encode_term(trs: TRS, t) -> np.ndarray:
    out: list[int] = []
    stack = [t]
    while stack:
        x = stack.pop()
        if x[0] == "$var":
            raise ParseError("input terms must be ground")
        out.append(trs.sym_id[x[0]])
        stack.extend(reversed(x[1]))
    return np.asarray(out, dtype=np.int32)


def decode_prefix(trs: TRS, codes) -> object:
    """Rebuild a nested-tuple term from a prefix code (iterative)."""
    codes = [int(c) for c in codes]
    if not codes:
        raise ParseError("empty code")
    root_holder: list = []
    stack = [(root_holder, 1)]
    for c in codes:
        if not stack:
            raise ParseError("trailing symbols in prefix code")
        kids: list = []
        node = (trs.symbols[c], kids)
        stack[-1][0].append(node)
        ar = trs.arity[c]
        if ar:
            stack.append((kids, ar))
        else:
            while stack and len(stack[-1][0]) == stack[-1][1]:
                stack.pop()
    if stack:
        raise ParseError("truncated prefix code")
    return root_holder[0]


def term_to_str(t) -> str:
    if t[0] == "$var":
        return t[1]
    out: list[str] = []
    stack: list = [t]
    while stack:
        x = stack.pop()
        if isinstance(x, str):
            out.append(x)
            continue
        if x[0] == "$var":
            out.append(x[1])
            continue
        if not x[1]:
            out.append(x[0])
            continue
        out.append(x[0] + "(")
        stack.append(")")
        for i, c in enumerate(reversed(x[1])):
            stack.append(c)
            if i != len(x[1]) - 1:
                stack.append(", ")
    return "".join(out)
