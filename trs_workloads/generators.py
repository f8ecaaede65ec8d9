"""Seeded generators for the five workload configurations.

Every generator returns a :class:`Workload`: the rewrite system, the ground
input terms as prefix codes (int32), the node-pool size and the maximum
arity.  Seeds: base 7174; configuration ``k`` uses ``7174 + k``; the batched
configurations derive one generator per term from ``(7177, i)``.

Recipes (the synthetic stand-ins for the paper's benchmark inputs, whose list
contents the paper elides):

* cfg0 - one complete binary plus/times tree with 1024 leaves (depth 10).
  Leaves are numerals ``S^k(0)`` with ``k`` uniform in 0..4.  Exactly
  ``floor((L-1)/10)`` of the internal nodes that sit at most two levels above
  the leaves become ``times`` (chosen uniformly among those), the rest
  ``plus``.  Pool 2^20 slots, maxarity 2.
* cfg1 - ``g(S^n(0))`` for n in {20, 25, 30}.  Pool 2^24, maxarity 2.
* cfg2 - ``sort(cons(v1, ... cons(v4096, nil)))`` with ``v`` uniform in
  0..63.  Pool 2^25, maxarity 3.
* cfg3 - 4096 independent terms; term ``i`` has kind ``i mod 3``: a plus/times
  tree with log-uniform size ``s`` in [1e2, 1e5] initial nodes and
  ``L = max(2, round(s/4))`` leaves, balanced by recursive halving; ``g(S^n(0))``
  with ``n`` uniform in 10..22; or ``sort`` of a list whose length is uniform in
  16..1024 with values uniform in 0..63.  Pool 2^27, maxarity 3.
* cfg4 - cfg3 plus ``g(S^32(0))`` (4097 terms).  Pool 2^27, maxarity 3.
* transformation tree of depth d - ``Expand(S^d(0))``.  Pool 2^26.
* tree merge sort "d k" - one complete binary ``Node`` tree of depth d whose
  2^d leaves are ``Leaf(Sort(list))`` of k numerals, values uniform in 0..9
  (seed 7174 + 6), in the paper's own merge-sort system (``Merge2`` of arity
  5).  Pool: the next power of two above four times the initial nodes, at
  most 2^30.

No function here rewrites, matches or evaluates a term.
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import systems
from .trs_text import TRS

BASE_SEED = 7174


@dataclass
class Workload:
    name: str
    trs: TRS
    terms: list                      # list of np.ndarray(int32) prefix codes
    pool_slots: int
    maxarity: int
    kinds: list = field(default_factory=list)   # per-term kind tag
    params: list = field(default_factory=list)  # per-term generator params

    @property
    def n_terms(self) -> int:
        return len(self.terms)

    @property
    def initial_nodes(self) -> int:
        return int(sum(len(t) for t in self.terms))

    def packed(self):
        """``(term_off int64[T+1], term_code int32[...])`` for the C-ABI."""
        off = np.zeros(len(self.terms) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(t) for t in self.terms])
        code = (np.concatenate(self.terms).astype(np.int32, copy=False)
                if self.terms else np.zeros(0, np.int32))
        return off, code


# --------------------------------------------------------------------------
# term builders (prefix codes)

def numeral(trs: TRS, k: int) -> np.ndarray:
    out = np.full(k + 1, trs.sym_id["S"], dtype=np.int32)
    out[-1] = trs.sym_id["0"]
    return out


def g_term(trs: TRS, n: int) -> np.ndarray:
    return np.concatenate([[trs.sym_id["g"]], numeral(trs, n)]).astype(np.int32)


def list_code(trs: TRS, values) -> np.ndarray:
    """``cons(v1, cons(v2, ... nil))`` with each value a numeral."""
    values = np.asarray(values, dtype=np.int64)
    S, Z = trs.sym_id["S"], trs.sym_id["0"]
    cons, nil = trs.sym_id["cons"], trs.sym_id["nil"]
    blk = values + 2                      # cons, S^v, 0
    total = int(blk.sum()) + 1
    out = np.full(total, S, dtype=np.int32)
    starts = np.zeros(len(values), dtype=np.int64)
    if len(values):
        starts[1:] = np.cumsum(blk)[:-1]
    out[starts] = cons
    out[starts + blk - 1] = Z
    out[-1] = nil
    return out


def sort_term(trs: TRS, values) -> np.ndarray:
    return np.concatenate([[trs.sym_id["sort"]], list_code(trs, values)]).astype(np.int32)


def peano_tree(trs: TRS, rng: np.random.Generator, n_leaves: int,
               leaf_max: int = 4) -> np.ndarray:
    """Balanced plus/times tree by recursive halving (left half gets the
    larger part).  RNG draw order: leaf values, then the times positions."""
    L = int(n_leaves)
    if L < 1:
        raise ValueError("need at least one leaf")
    leaves = rng.integers(0, leaf_max + 1, size=L)
    # internal nodes in prefix order: (leftmost leaf, number of leaves)
    left_leaf: list[int] = []
    size: list[int] = []
    stack = [(0, L)]
    while stack:
        lo, m = stack.pop()
        if m == 1:
            continue
        left_leaf.append(lo)
        size.append(m)
        h = (m + 1) // 2
        stack.append((lo + h, m - h))     # right pushed first
        stack.append((lo, h))
    left_leaf_a = np.asarray(left_leaf, dtype=np.int64)
    size_a = np.asarray(size, dtype=np.int64)
    # height of a recursive-halving subtree with m leaves is ceil(log2 m);
    # "at most two levels above the leaves" means m <= 4
    eligible = np.nonzero(size_a <= 4)[0]
    k = min((L - 1) // 10, len(eligible))
    ops = np.full(len(size_a), trs.sym_id["plus"], dtype=np.int32)
    if k:
        pick = rng.choice(len(eligible), size=k, replace=False)
        ops[eligible[pick]] = trs.sym_id["times"]
    # assemble: before leaf j come the internal nodes whose leftmost leaf is j
    run = np.bincount(left_leaf_a, minlength=L) if len(left_leaf_a) else np.zeros(L, np.int64)
    blk = run + leaves + 1
    total = int(blk.sum())
    out = np.full(total, trs.sym_id["S"], dtype=np.int32)
    starts = np.zeros(L, dtype=np.int64)
    starts[1:] = np.cumsum(blk)[:-1]
    # internal node positions: internal nodes are already grouped by leftmost
    # leaf in prefix order, top-down inside a group
    if len(ops):
        grp_start = np.repeat(starts, run)
        first_of_grp = np.zeros(L, dtype=np.int64)
        first_of_grp[1:] = np.cumsum(run)[:-1]
        within = np.arange(len(ops)) - np.repeat(first_of_grp, run)
        out[grp_start + within] = ops
    out[starts + blk - 1] = trs.sym_id["0"]
    return out


# --------------------------------------------------------------------------
# configurations

def cfg0(seed: int = BASE_SEED + 0) -> Workload:
    trs = systems.peano()
    rng = np.random.default_rng(seed)
    t = peano_tree(trs, rng, 1024)
    return Workload("cfg0_peano_tree_1024", trs, [t], 1 << 20, 2,
                    kinds=["peano"], params=[{"leaves": 1024}])


def cfg1(n: int = 20) -> Workload:
    trs = systems.fib()
    return Workload(f"cfg1_fib_g{n}", trs, [g_term(trs, n)], 1 << 24, 2,
                    kinds=["g"], params=[{"n": n}])


def cfg2(length: int = 4096, seed: int = BASE_SEED + 2) -> Workload:
    trs = systems.msort()
    rng = np.random.default_rng(seed)
    vals = rng.integers(0, 64, size=length)
    return Workload(f"cfg2_msort_{length}", trs, [sort_term(trs, vals)], 1 << 25, 3,
                    kinds=["sort"], params=[{"len": length}])


def _batch_term(trs: TRS, i: int, size_lo=1e2, size_hi=1e5, g_lo=10, g_hi=22,
                len_lo=16, len_hi=1024):
    rng = np.random.default_rng([BASE_SEED + 3, i])
    kind = i % 3
    if kind == 0:
        s = math.exp(rng.uniform(math.log(size_lo), math.log(size_hi)))
        L = max(2, int(round(s / 4)))
        return "peano", {"leaves": L}, peano_tree(trs, rng, L)
    if kind == 1:
        n = int(rng.integers(g_lo, g_hi + 1))
        return "g", {"n": n}, g_term(trs, n)
    ln = int(rng.integers(len_lo, len_hi + 1))
    vals = rng.integers(0, 64, size=ln)
    return "sort", {"len": ln}, sort_term(trs, vals)


_CACHE: dict = {}


def cfg3(n_terms: int = 4096, pool_slots: int = 1 << 27, scale: str = "full") -> Workload:
    """``scale='mini'`` keeps the recipe but shrinks every size range (for
    tests the oracle must finish quickly)."""
    key = ("cfg3", n_terms, pool_slots, scale)
    if key in _CACHE:
        return _CACHE[key]
    trs = systems.batch()
    if scale == "full":
        rng_args = {}
    elif scale == "mini":
        rng_args = dict(size_lo=1e1, size_hi=2e3, g_lo=2, g_hi=14, len_lo=0, len_hi=64)
    else:
        raise ValueError(scale)
    terms, kinds, params = [], [], []
    for i in range(n_terms):
        k, p, t = _batch_term(trs, i, **rng_args)
        terms.append(t)
        kinds.append(k)
        params.append(p)
    w = Workload(f"cfg3_batch_{n_terms}" + ("" if scale == "full" else "_" + scale),
                 trs, terms, pool_slots, 3, kinds, params)
    _CACHE[key] = w
    return w


def cfg4(n_terms: int = 4096, pool_slots: int = 1 << 27, scale: str = "full",
         g_big: int = 32) -> Workload:
    base = cfg3(n_terms, pool_slots, scale)
    trs = base.trs
    return Workload(f"cfg4_batch_{n_terms}_g{g_big}" + ("" if scale == "full" else "_" + scale),
                    trs, base.terms + [g_term(trs, g_big)], pool_slots, 3,
                    base.kinds + ["g"], base.params + [{"n": g_big}])


def ttree(depth: int = 22, pool_slots: int = 1 << 26) -> Workload:
    trs = systems.ttree()
    t = np.concatenate([[trs.sym_id["Expand"]], numeral(trs, depth)]).astype(np.int32)
    return Workload(f"ttree_{depth}", trs, [t], pool_slots, 2,
                    kinds=["ttree"], params=[{"depth": depth}])


def tmsort(depth: int = 23, length: int = 5, seed: int = BASE_SEED + 6, vmax: int = 9,
           pool_slots: int = 0) -> Workload:
    """Tree merge sort: ``Node`` tree of depth ``depth`` over 2^depth leaves
    ``Leaf(Sort(Cons(S^v1(Zero), ... Nil)))`` of ``length`` values each.

    In prefix order leaf 0 follows ``depth`` Node symbols and leaf i > 0
    follows as many as i has trailing zero bits (the subtrees it starts)."""
    trs = systems.msort5()
    sid = trs.sym_id
    L = 1 << depth
    vals = np.random.default_rng(seed).integers(0, vmax + 1, size=(L, length))
    i = np.arange(L, dtype=np.int64)
    k = np.zeros(L, dtype=np.int64)
    k[0] = depth
    low = i[1:] & -i[1:]                                   # lowest set bit
    k[1:] = np.log2(low).astype(np.int64)
    blk = vals + 2                                          # Cons, S^v, Zero
    leaf_len = 3 + blk.sum(axis=1)                          # Leaf, Sort, ..., Nil
    start = np.zeros(L, dtype=np.int64)
    start[1:] = np.cumsum(k + leaf_len)[:-1]
    total = int((k + leaf_len).sum())
    out = np.full(total, sid["S"], dtype=np.int32)
    run = np.repeat(np.cumsum(k) - k, k)
    out[np.repeat(start, k) + np.arange(int(k.sum())) - run] = sid["Node"]
    p = start + k
    out[p] = sid["Leaf"]
    out[p + 1] = sid["Sort"]
    bstart = p[:, None] + 2 + np.concatenate(
        [np.zeros((L, 1), np.int64), np.cumsum(blk, axis=1)[:, :-1]], axis=1)
    out[bstart] = sid["Cons"]
    out[bstart + 1 + vals] = sid["Zero"]
    out[p + leaf_len - 1] = sid["Nil"]
    if not pool_slots:  # (the library takes at most 2^30 slots)
        pool_slots = 1 << min(30, max(20, int(math.ceil(math.log2(4 * total)))))
    return Workload(f"tmsort_{depth}_{length}", trs, [out], pool_slots, 5,
                    kinds=["tmsort"], params=[{"depth": depth, "length": length}])


def cache_path() -> str:
    return os.environ.get("TRS_WORKLOAD_CACHE", "/tmp/trs_workloads_cache")
