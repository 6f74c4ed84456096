"""Oracle, part 2: counting quantifiers of LTL4-C over a finite trace.

TEST INFRASTRUCTURE ONLY (see the header of oracle/ltl.py).

What it computes, section by section of the paper:
* the value vectors of a trace (Section 2.4.1, Eq. 5): one vector per event,
  made of the values its key fields carry for the quantified variables;
* the clusters u^D (Section 2.4.3): the events carrying vector D, in trace
  order;
* the leaf verdicts [u^D |=4 psi] (Def. 5), from a caller-supplied leaf
  function (the tableau of oracle/ltl.py, or a monitor table);
* P (Section 2.4.2), B and S (Section 2.4.3-2.4.4, Eq. 6) and the inductive
  semantics of Def. 7, applied from the innermost quantifier outwards as the
  quantifier submonitors of Def. 8 do (Section 3.4).

Readings (each one is listed in the design notes):
* Def. 7's presumably-false case requires S(B6 - {F, Fc}) = 0, which would
  make it coincide with currently-false; it is read as "= 1", which is what
  the informal description of presumably false in Section 2.3 says.
* Where several cases of Def. 7 hold, the one highest in the B6 lattice wins
  (Section 2.3 says Tc and Tp take precedence over lower values).
* The clauses "for every extension the verdict stays T / F" are read in the
  abstract extension model: children that are T or F keep that verdict, every
  other child may end up satisfied or violated, and any number of new children
  of either kind may appear.  `perm_sat` / `perm_viol` are the closed forms of
  that model; they contain Table 1 and the rule for the default A=1 verbatim.
  tests/test_oracle_counting.py checks them against an enumeration of
  extensions.
* Percentage constants are exact rationals num/den (0.95 = 19/20); instance
  counts are integers >= 0.
* With no children (N = 0) the same rules apply with all counts zero.
* An event that lacks the key of any quantifier joins no cluster.
* Parent events (an option; the proxy-cache case study of Section 5 observes
  per-video events in every request of the video): an event that carries the
  values of x_0..x_{n-2} but none for x_{n-1} joins u^D for every D in the set
  of value vectors (Eq. 5) whose first n-1 values are its own, at its trace
  position.  It adds no vector to that set, so it makes no instance and no
  node.  For a single quantifier this is an event with no key, which joins
  every cluster.
"""
from __future__ import annotations

from fractions import Fraction

from .ltl import BOT, BOT_C, BOT_P, TOP_P, TOP_C, TOP

PERCENT, COUNT = "A", "E"          # the percentage and instance-counting quantifiers
OPS = ("<", "<=", ">", ">=", "=")


def compare(lhs, op, rhs):
    if op == "<":
        return lhs < rhs
    if op == "<=":
        return lhs <= rhs
    if op == ">":
        return lhs > rhs
    if op == ">=":
        return lhs >= rhs
    if op == "=":
        return lhs == rhs
    raise ValueError(op)


def constraint(kind, op, const, k, n):
    """Eq. 6: S for a set of children of size k out of n children."""
    if kind == PERCENT:
        return compare(Fraction(k), op, Fraction(const) * n)
    return compare(k, op, const)


def perm_sat(kind, op, const, v):
    """No extension can make the count of T children fail the constraint."""
    k_top = v[TOP]
    c = Fraction(const)
    if kind == COUNT:
        if op in (">", ">="):          # Table 1, rows > and >=
            return compare(k_top, op, const)
        return False
    v_bot = v[BOT]
    if op == ">=":
        return c == 0
    if op == ">":
        return c == 0 and k_top >= 1
    if op == "<=":
        return c == 1
    if op == "<":
        return c == 1 and v_bot >= 1
    return False                       # "=": some extension always breaks it


def perm_viol(kind, op, const, v):
    """No extension can make the count of non-F children meet the constraint."""
    k_top = v[TOP]
    c = Fraction(const)
    if kind == COUNT:
        if op in ("=", "<="):          # Table 1: violation once the count exceeds l
            return k_top > const
        if op == "<":                  # Table 1: violation once the count reaches l
            return k_top >= const
        return False
    v_bot = v[BOT]
    if op == ">=":
        return c == 1 and v_bot >= 1   # the default A=1: one F child violates it for good
    if op == ">":
        return c == 1
    if op == "<=":
        return c == 0 and k_top >= 1
    if op == "<":
        return c == 0
    return (c == 1 and v_bot >= 1) or (c == 0 and k_top >= 1)   # "="


def valuate(kind, op, const, v):
    """Def. 7 for one quantifier submonitor with child-verdict counts v[0..5]."""
    n = sum(v)
    # the nested sets of truth values Def. 7 applies S to
    k1 = v[TOP]                                     # {T}
    k2 = k1 + v[TOP_C]                              # {T, Tc}
    k3 = k2 + v[TOP_P]                              # {T, Tc, Tp}
    k4 = k3 + v[BOT_P]                              # B6 - {F, Fc}
    k5 = k4 + v[BOT_C]                              # B6 - {F}
    s = lambda k: constraint(kind, op, const, k, n)
    if s(k1) and perm_sat(kind, op, const, v):
        return TOP
    if s(k2):
        return TOP_C
    if s(k3):
        return TOP_P
    if s(k4):
        return BOT_P
    if not s(k5) and perm_viol(kind, op, const, v):
        return BOT
    return BOT_C


def evaluate(events, quants, leaf, parent_events=False):
    """Evaluate phi = Q_0 ... Q_{n-1} psi on a trace.

    events : sequence of (letter, key) in trace order; key is a tuple of the n
             values the event carries for x_0..x_{n-1}, or None when the event
             lacks one of them.  With parent_events, a key of n-1 values marks
             a parent event (see the module header).
    quants : [(kind, op, const)] for Q_0 .. Q_{n-1}.
    leaf   : function from a non-empty list of letters (a cluster, in trace
             order) to its LTL4 verdict.
    Returns (root_verdict, nodes, leaves) where
      leaves[D] = verdict of the instance with full vector D,
      nodes[prefix] = (counts v, verdict) for every partial vector of length
      0 .. n-1 that occurs (the root is the empty tuple).
    """
    n = len(quants)
    clusters = {}
    for letter, key in events:
        if key is None:
            continue
        if len(key) == n - 1 and parent_events:
            continue
        if len(key) != n:
            raise ValueError("key length must equal the number of quantifiers")
        clusters.setdefault(tuple(key), []).append(letter)
    if parent_events:
        # u^D written out: every event, in trace order, whose values are D's
        # or, for a parent event, the first n-1 of D's
        for d in clusters:
            clusters[d] = [letter for letter, key in events
                           if key is not None and (tuple(key) == d or (len(key) == n - 1 and tuple(key) == d[:n - 1]))]
    verdict = {d: leaf(word) for d, word in clusters.items()}
    leaves = dict(verdict)
    nodes = {}
    level = verdict                      # verdicts of the partial vectors of length m+1
    for m in range(n - 1, -1, -1):
        children = {}
        for d, b in level.items():
            children.setdefault(d[:m], []).append(b)
        if m == 0 and not children:
            children[()] = []            # the root exists even with no instances
        nxt = {}
        for prefix, bs in children.items():
            v = [0] * 6
            for b in bs:
                v[b] += 1
            kind, op, const = quants[m]
            r = valuate(kind, op, const, v)
            nodes[prefix] = (v, r)
            nxt[prefix] = r
        level = nxt
    return level[()], nodes, leaves
